"""Python binding of libdust, the gfx950 dust-temperature library.

Argument marshalling only: every step of the calculation runs in the HIP
kernels of ``libdust.so`` behind the C-ABI declared in ``include/dust.h``.
torch tensors serve as device buffers (their data pointers and the current
HIP stream are passed through).  There is no CPU fallback: if the library is
not built, or no GPU is present, calls raise.

Section 4 of Jonsson & Primack (New Astronomy, "Accelerating Dust Temperature
Calculations with Graphics Processing Units") defines the three steps:
absorb (Eq. 6), solve (Eq. 7) and emit (Eqs. 9-10).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdust.so")

DUST_OK, DUST_EINVAL, DUST_EUNSUPPORTED, DUST_ENOMEM, DUST_EDEVICE = 0, -1, -2, -3, -4
PLAIN, MIXED, TABLE_LINEAR = 0, 1, 2
BATCH_AUTOTUNE, BATCH_REFRESH_PLANS = 1, 2
_MODES = {"plain": PLAIN, "mixed": MIXED, "table": TABLE_LINEAR,
          PLAIN: PLAIN, MIXED: MIXED, TABLE_LINEAR: TABLE_LINEAR}
N_COUNTERS = 4  # nonfinite, unconverged, out_of_table, newton_evals

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class GridDesc(ctypes.Structure):
    _fields_ = [("n_lambda", _i32), ("n_grains", _i32),
                ("lambda_", _vp), ("dlambda", _vp), ("c_abs", _vp),
                ("weight", _vp), ("size", _vp)]


class Options(ctypes.Structure):
    _fields_ = [("mode", _i32), ("maxit", _i32), ("tol", ctypes.c_double),
                ("ltab_n", _i32), ("fused_kernels", _i32),
                ("ltab_tmin", ctypes.c_double), ("ltab_tmax", ctypes.c_double),
                ("f32_lookup", _i32), ("newton_polish", _i32), ("reserved", _i32)]


class Levels(ctypes.Structure):
    _fields_ = [("n_levels", _i32), ("T", _vp), ("E", _vp)]


class SolveExt(ctypes.Structure):
    _fields_ = [("Q", _vp), ("ldq", _i64), ("warm_start", _i32), ("reserved", _i32)]


class DustError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdust error {code}: {msg}")
        self.code = code


_lib = None


def build():
    """Compile libdust.so in-tree (hipcc, gfx950)."""
    from . import builder
    return builder.build()


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_0907_3768_amd.build()")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    L.dust_last_error.restype = ctypes.c_char_p
    L.dust_version.restype = ctypes.c_char_p
    sigs = {
        "dust_plan_create": [ctypes.POINTER(GridDesc), ctypes.POINTER(Options), ctypes.POINTER(_vp)],
        "dust_plan_destroy": [_vp],
        "dust_plan_prepare": [_vp, _vp],
        "dust_plan_info": [_vp, _vp, _vp, _vp],
        "dust_absorb": [_vp, _i64, _vp, _i64, _vp, _i64, _vp],
        "dust_solve_T": [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp],
        "dust_solve_T_ext": [_vp, _i64, _vp, _i64, ctypes.POINTER(SolveExt), _vp, _i64, _vp, _vp],
        "dust_emit_sed": [_vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp],
        "dust_run_fused": [_vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _vp],
        "dust_run_fused_ext": [_vp, _i64, _vp, _i64, _vp, ctypes.POINTER(SolveExt), _vp, _i64,
                               _vp, _i64, _vp, _vp],
        "dust_batch_create": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32,
                              ctypes.POINTER(_vp)],
        "dust_batch_launch": [_vp, _vp],
        "dust_batch_info": [_vp, _vp, _vp],
        "dust_batch_form": [_vp, _vp, _vp, _vp],
        "dust_batch_destroy": [_vp],
        "dust_batch_run": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
        "dust_batch_run_noalloc": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp],
        "dust_fluct_plan_create": [ctypes.POINTER(GridDesc), ctypes.POINTER(Levels),
                                   ctypes.POINTER(_vp)],
        "dust_fluct_plan_destroy": [_vp],
        "dust_fluct_solve_P": [_vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp],
        "dust_fluct_emit_sed": [_vp, _i64, _vp, _i64, _vp, _vp, _i64, _i32, _vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.restype = st
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().dust_last_error().decode()


def _check(code):
    if code != DUST_OK:
        raise DustError(code, last_error())


def _stream(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _on_device(t, name, device):
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the plan on cuda:{device}")


def _rows(t, width, name, rows=None, device=None):
    """(pointer, leading dimension) of a 2-D float32 CUDA tensor with unit column
    stride, at least `width` columns and at least `rows` rows: the kernels
    touch rows 0 .. rows - 1 of it, so a shorter tensor is refused here."""
    import torch
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if t.dim() != 2 or t.stride(1) != 1 or t.shape[1] < width:
        raise ValueError(f"{name} must be 2-D, row-major, with at least {width} columns")
    if rows is not None and t.shape[0] < rows:
        raise ValueError(f"{name} has {t.shape[0]} rows, the call needs {rows}")
    _on_device(t, name, device)
    return _vp(t.data_ptr()), t.stride(0) if t.shape[0] > 1 else max(t.shape[1], width)


def _vec(t, n, name, dtype, device=None):
    """Pointer of a contiguous CUDA tensor of `dtype` with at least n elements,
    or NULL for None."""
    if t is None:
        return _vp(0)
    if t.dtype != dtype or not t.is_cuda:
        raise TypeError(f"{name} must be a {dtype} CUDA tensor")
    if not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{name} must be contiguous with at least {n} elements")
    _on_device(t, name, device)
    return _vp(t.data_ptr())


def _masses(m_dust, n, device=None):
    import torch
    return _vec(m_dust, n, "m_dust", torch.float32, device)


def _counters(counters, device=None):
    import torch
    return _vec(counters, N_COUNTERS, "counters", torch.int64, device)


def new_counters(device="cuda"):
    """A zeroed device dust_counters (int64 x 4: nonfinite, unconverged,
    out_of_table, newton_evals)."""
    import torch
    return torch.zeros(N_COUNTERS, dtype=torch.int64, device=device)


def _ext(Q, warm_start, width, rows, device=None):
    """A dust_solve_ext for (Q, warm_start), or None when neither is given."""
    if Q is None and not warm_start:
        return None
    if Q is None:
        return SolveExt(None, 0, 1, 0)
    pq, ldq = _rows(Q, width, "Q", rows, device)
    return SolveExt(pq, ldq, 1 if warm_start else 0, 0)


class Plan:
    """A grid's device tables (dust_plan)."""

    def __init__(self, grid, mode="plain", tol=0.0, maxit=0, ltab_n=0, ltab_tmin=0.0,
                 ltab_tmax=0.0, fused_kernels=0, f32_lookup=False, newton_polish=False):
        self._keep = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (grid.lam, grid.dlam, grid.c_abs, grid.weight, grid.size)]
        lam, dlam, cabs, w, a = self._keep
        self.n_lambda = int(lam.shape[0])
        self.n_grains = int(cabs.shape[0])
        self.mode = _MODES[mode]
        desc = GridDesc(self.n_lambda, self.n_grains, lam.ctypes.data, dlam.ctypes.data,
                        cabs.ctypes.data, w.ctypes.data, a.ctypes.data)
        opt = Options(self.mode, int(maxit), float(tol), int(ltab_n), int(fused_kernels),
                      float(ltab_tmin), float(ltab_tmax), 1 if f32_lookup else 0,
                      1 if newton_polish else 0, 0)
        h = _vp()
        _check(lib().dust_plan_create(ctypes.byref(desc), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        import torch
        self.device = torch.cuda.current_device()  # the plan's tables live there

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dust_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, stream=None):
        _check(lib().dust_plan_prepare(self._h, _stream(stream)))

    def _alloc(self, n, width, like):
        import torch
        return torch.empty((n, width), dtype=torch.float32, device=like.device)

    def absorb(self, J, H=None, stream=None):
        n = J.shape[0]
        H = self._alloc(n, self.n_grains, J) if H is None else H
        pj, ldj = _rows(J, self.n_lambda, "J", n, self.device)
        ph, ldh = _rows(H, self.n_grains, "H", n, self.device)
        _check(lib().dust_absorb(self._h, n, pj, ldj, ph, ldh, _stream(stream)))
        return H

    def solve(self, H, T=None, counters=None, stream=None, Q=None, warm_start=False):
        """Eq. 7 for every pair.  Q: extra heating added to H; warm_start: T
        already holds a previous solution, where the plain Newton starts."""
        n = H.shape[0]
        if warm_start and T is None:
            raise ValueError("warm_start needs T holding the previous temperatures")
        T = self._alloc(n, self.n_grains, H) if T is None else T
        ph, ldh = _rows(H, self.n_grains, "H", n, self.device)
        pt, ldt = _rows(T, self.n_grains, "T", n, self.device)
        x = _ext(Q, warm_start, self.n_grains, n, self.device)
        pc = _counters(counters, self.device)
        if x is None:
            _check(lib().dust_solve_T(self._h, n, ph, ldh, pt, ldt, pc, _stream(stream)))
        else:
            _check(lib().dust_solve_T_ext(self._h, n, ph, ldh, ctypes.byref(x), pt, ldt, pc,
                                          _stream(stream)))
        return T

    def emit(self, T, m_dust=None, L=None, stream=None):
        n = T.shape[0]
        L = self._alloc(n, self.n_lambda, T) if L is None else L
        pt, ldt = _rows(T, self.n_grains, "T", n, self.device)
        pl, ldl = _rows(L, self.n_lambda, "L", n, self.device)
        pm = _masses(m_dust, n, self.device)
        _check(lib().dust_emit_sed(self._h, n, pt, ldt, pm, pl, ldl, _stream(stream)))
        return L

    def fused(self, J, m_dust=None, T=None, L=None, counters=None, stream=None, Q=None,
              warm_start=False):
        """absorb -> solve -> emit in one launch per tile; Q and warm_start as
        in ``solve``."""
        n = J.shape[0]
        if warm_start and T is None:
            raise ValueError("warm_start needs T holding the previous temperatures")
        T = self._alloc(n, self.n_grains, J) if T is None else T
        L = self._alloc(n, self.n_lambda, J) if L is None else L
        pj, ldj = _rows(J, self.n_lambda, "J", n, self.device)
        pt, ldt = _rows(T, self.n_grains, "T", n, self.device)
        pl, ldl = _rows(L, self.n_lambda, "L", n, self.device)
        pm = _masses(m_dust, n, self.device)
        pc = _counters(counters, self.device)
        x = _ext(Q, warm_start, self.n_grains, n, self.device)
        if x is None:
            _check(lib().dust_run_fused(self._h, n, pj, ldj, pm, pt, ldt, pl, ldl, pc,
                                        _stream(stream)))
        else:
            _check(lib().dust_run_fused_ext(self._h, n, pj, ldj, pm, ctypes.byref(x),
                                            pt, ldt, pl, ldl, pc, _stream(stream)))
        return T, L

    def run(self, J, m_dust=None, counters=None, stream=None, Q=None, T=None,
            warm_start=False):
        """absorb -> solve -> emit as three launches; returns (H, T, L)."""
        H = self.absorb(J, stream=stream)
        T = self.solve(H, T=T, counters=counters, stream=stream, Q=Q, warm_start=warm_start)
        L = self.emit(T, m_dust, stream=stream)
        return H, T, L


class FluctPlan:
    """Thermally fluctuating grains of a grid (dust_fluct_plan): the level
    distributions P[c, s, j] and the emission averaged over them."""

    def __init__(self, grid, lev_T, lev_E):
        self._keep = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (grid.lam, grid.dlam, grid.c_abs, grid.weight, grid.size,
                                lev_T, lev_E)]
        lam, dlam, cabs, w, a, lt, le = self._keep
        self.n_lambda = int(lam.shape[0])
        self.n_grains = int(cabs.shape[0])
        if lt.ndim != 2 or lt.shape != le.shape or lt.shape[0] != self.n_grains:
            raise ValueError("lev_T and lev_E must both be [n_grains, n_levels]")
        self.n_levels = int(lt.shape[1])
        desc = GridDesc(self.n_lambda, self.n_grains, lam.ctypes.data, dlam.ctypes.data,
                        cabs.ctypes.data, w.ctypes.data, a.ctypes.data)
        lv = Levels(self.n_levels, lt.ctypes.data, le.ctypes.data)
        h = _vp()
        _check(lib().dust_fluct_plan_create(ctypes.byref(desc), ctypes.byref(lv),
                                            ctypes.byref(h)))
        self._h = h
        import torch
        self.device = torch.cuda.current_device()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dust_fluct_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_P(self, J, P=None, counters=None, stream=None):
        """P[c, s * n_levels + j] (float32 [C, >= S M]) from J[C, NL]."""
        import torch
        n = J.shape[0]
        K = self.n_grains * self.n_levels
        if P is None:
            P = torch.empty((n, K), dtype=torch.float32, device=J.device)
        pj, ldj = _rows(J, self.n_lambda, "J", n, self.device)
        pp, ldp = _rows(P, K, "P", n, self.device)
        pc = _counters(counters, self.device)
        _check(lib().dust_fluct_solve_P(self._h, n, pj, ldj, pp, ldp, pc, _stream(stream)))
        return P

    def emit(self, P, m_dust=None, L=None, accumulate=False, stream=None):
        """L[c, l] from the distributions; accumulate adds onto L."""
        n = P.shape[0]
        K = self.n_grains * self.n_levels
        if L is None:
            if accumulate:
                raise ValueError("accumulate needs L")
            import torch
            L = torch.empty((n, self.n_lambda), dtype=torch.float32, device=P.device)
        pp, ldp = _rows(P, K, "P", n, self.device)
        pl, ldl = _rows(L, self.n_lambda, "L", n, self.device)
        pm = _masses(m_dust, n, self.device)
        _check(lib().dust_fluct_emit_sed(self._h, n, pp, ldp, pm, pl, ldl,
                                         1 if accumulate else 0, _stream(stream)))
        return L


def _grid_arrays(plans, J, m_dust, T, L):
    """The per-grid host arrays of a batched call, after the binding's checks
    (every tensor covers its grid's rows, on the plans' device)."""
    n = len(plans)
    arr = lambda typ, vals: (typ * n)(*vals)
    hp = arr(_vp, [p.handle.value for p in plans])
    nc = arr(_i64, [j.shape[0] for j in J])
    pj, ldj, pt, ldt, pl, ldl = [], [], [], [], [], []
    for p, j, t, l in zip(plans, J, T, L):
        rows = j.shape[0]
        a, b = _rows(j, p.n_lambda, "J", rows, p.device); pj.append(a.value or 0); ldj.append(b)
        a, b = _rows(t, p.n_grains, "T", rows, p.device); pt.append(a.value or 0); ldt.append(b)
        a, b = _rows(l, p.n_lambda, "L", rows, p.device); pl.append(a.value or 0); ldl.append(b)
    pm = [_masses(m, j.shape[0], p.device).value or 0 for p, m, j in zip(plans, m_dust, J)]
    return (hp, nc, arr(_vp, pj), arr(_i64, ldj), arr(_vp, pm), arr(_vp, pt),
            arr(_i64, ldt), arr(_vp, pl), arr(_i64, ldl))


def _as_vp(a):
    return [ctypes.cast(x, _vp) for x in a]


def batch_run(plans: Sequence[Plan], J, m_dust, T, L, counters=None, stream=None,
              no_alloc=False):
    """One-shot batched launch (dust_batch_run): absorb -> solve -> emit for
    every grid in one kernel, nothing kept.  no_alloc: dust_batch_run_noalloc
    (the work list in the library's fixed device array; calls that may
    overlap on one device race)."""
    if not (len(plans) == len(J) == len(m_dust) == len(T) == len(L)):
        raise ValueError("plans, J, m_dust, T and L must have one entry per grid")
    a = _grid_arrays(plans, J, m_dust, T, L)
    pc = _counters(counters, plans[0].device if plans else None)
    v = _as_vp(a)
    f = lib().dust_batch_run_noalloc if no_alloc else lib().dust_batch_run
    _check(f(v[0], len(plans), v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], pc,
             _stream(stream)))


class Batch:
    """Many grids in one launch recorded in a HIP graph (dust_batch)."""

    def __init__(self, plans: Sequence[Plan], J, m_dust, T, L, counters=None, autotune=True,
                 refresh_plans=False):
        if not (len(plans) == len(J) == len(m_dust) == len(T) == len(L)):
            raise ValueError("plans, J, m_dust, T and L must have one entry per grid")
        self._plans = list(plans)
        self._bufs = (list(J), list(m_dust), list(T), list(L), counters)
        self._arrays = _grid_arrays(plans, J, m_dust, T, L)
        pc = _counters(counters, plans[0].device if plans else None)
        h = _vp()
        v = _as_vp(self._arrays)
        _check(lib().dust_batch_create(v[0], len(plans), v[1], v[2], v[3], v[4], v[5], v[6],
                                       v[7], v[8], pc,
                                       (BATCH_AUTOTUNE if autotune else 0) |
                                       (BATCH_REFRESH_PLANS if refresh_plans else 0),
                                       ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().dust_batch_launch(self._h, _stream(stream)))

    def info(self):
        tc = _i32()
        ni = _i64()
        _check(lib().dust_batch_info(self._h, ctypes.byref(tc), ctypes.byref(ni)))
        return {"cells_per_tile": tc.value, "n_items": ni.value}

    def form(self):
        """(cells per tile, grain tiles per wave, work-queue workgroups per CU
        or 0 for one workgroup per item)."""
        tc, ntw, pc = _i32(), _i32(), _i32()
        _check(lib().dust_batch_form(self._h, ctypes.byref(tc), ctypes.byref(ntw),
                                     ctypes.byref(pc)))
        return tc.value, ntw.value, pc.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dust_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
