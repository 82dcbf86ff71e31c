"""FP64 CPU oracle for the dust equilibrium-temperature and emission path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product package never does.  It shares
no code, header, table or constant with the GPU path.

The arithmetic lives in ``dust_ref.c`` (plain C, IEEE double precision, one
function per equation of Section 4: Eq. 6 heating, Eq. 7 temperature root,
Eqs. 9-10 emission, Eq. 11 initial guess, and the production variant of the
temperature step: linear interpolation in a table of the grain power) and
``fluct_ref.c`` (thermally fluctuating grains, Sections 2 and 6: the level
distribution under single-photon heating and continuous cooling, and the
emission averaged over it).  This
module builds that file with gcc, marshals numpy arrays to it, and adds the
non-radiative heating term and the outer re-heating iteration (Section 2) as
plain numpy around those calls.

Every function is pinned by tests against what physics and mathematics fix
(Stefan-Boltzmann, Wien displacement, grey and power-law grains in diluted
blackbody fields, brute-force bisection, the SED energy identity, BLAS for
the heating product, numpy's piecewise-linear interpolation for the table
variant, closed forms for the extra heating and the re-heating series).  The Eq. 11 guess is not pinned to any value (the
paper prints none for the grains used here); it only changes how many
iterations the solve takes, never the root, and a test checks exactly that.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dust_ref.c")
_SRC_FLUCT = os.path.join(_HERE, "fluct_ref.c")
_LIB_PATH = os.path.join(_HERE, "libdust_ref.so")
_lib = None

_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile dust_ref.c into libdust_ref.so (gcc, OpenMP, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, _SRC_FLUCT, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.dust_ref_planck.restype = _d
        L.dust_ref_planck.argtypes = [_d, _d]
        L.dust_ref_planck_dT.restype = _d
        L.dust_ref_planck_dT.argtypes = [_d, _d]
        L.dust_ref_grain_power.restype = _d
        L.dust_ref_grain_power.argtypes = [_i32, _p, _p, _p, _d]
        L.dust_ref_guess.restype = _d
        L.dust_ref_guess.argtypes = [_d, _d]
        L.dust_ref_heating.restype = None
        L.dust_ref_heating.argtypes = [_i64, _i32, _i32, _p, _i64, _p, _p, _p]
        L.dust_ref_temperature.restype = None
        L.dust_ref_temperature.argtypes = [_i64, _i32, _i32, _p, _p, _p, _p, _p, _p, _p]
        L.dust_ref_emission.restype = None
        L.dust_ref_emission.argtypes = [_i64, _i32, _i32, _p, _p, _p, _p, _p, _p]
        L.dust_ref_table_build.restype = None
        L.dust_ref_table_build.argtypes = [_i32, _i32, _p, _p, _p, _i32, _d, _d, _p]
        L.dust_ref_table_temperature.restype = _i64
        L.dust_ref_table_temperature.argtypes = [_i64, _i32, _i32, _d, _d, _p, _p, _p]
        L.dust_ref_fluct_pair.restype = None
        L.dust_ref_fluct_pair.argtypes = [_i32, _i32, _p, _p, _p, _p, _p, _p, _p]
        L.dust_ref_fluct_distribution.restype = None
        L.dust_ref_fluct_distribution.argtypes = [_i64, _i32, _i32, _i32, _p, _p, _p, _p, _p,
                                                  _p, _i64, _p]
        L.dust_ref_fluct_emission.restype = None
        L.dust_ref_fluct_emission.argtypes = [_i64, _i32, _i32, _i32, _p, _p, _p, _p, _p, _p,
                                              _p]
        L.dust_ref_get_threads.restype = ctypes.c_int
        L.dust_ref_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def planck(lam, T):
    """B_lambda(lam, T) (scalar or array, element-wise)."""
    f = np.vectorize(lambda x, t: lib().dust_ref_planck(float(x), float(t)))
    return f(lam, T)


def planck_dT(lam, T):
    f = np.vectorize(lambda x, t: lib().dust_ref_planck_dT(float(x), float(t)))
    return f(lam, T)


def grain_power(lam, dlam, c_row, T):
    """sum_l C[l] dlam[l] B(lam_l, T), the right side of Eq. 7."""
    lam, dlam, c_row = _f64(lam), _f64(dlam), _f64(c_row)
    return lib().dust_ref_grain_power(lam.shape[0], _ptr(lam), _ptr(dlam), _ptr(c_row), float(T))


def guess(lh_watt, a_m):
    """Eq. 11 initial guess (K) for heating luminosity ``lh_watt`` and size ``a_m``."""
    f = np.vectorize(lambda x, a: lib().dust_ref_guess(float(x), float(a)))
    return f(lh_watt, a_m)


def heating(J, c_abs, dlam):
    """Eq. 6: H[C,S] from J[C,NL] (any float dtype, upcast), C_abs[S,NL], dlam[NL]."""
    J = _f64(J)
    c_abs, dlam = _f64(c_abs), _f64(dlam)
    C, NL = J.shape
    S = c_abs.shape[0]
    assert c_abs.shape == (S, NL) and dlam.shape == (NL,)
    H = np.empty((C, S), dtype=np.float64)
    lib().dust_ref_heating(C, NL, S, _ptr(J), NL, _ptr(c_abs), _ptr(dlam), _ptr(H))
    return H


def temperature(H, lam, dlam, c_abs, size, return_iters=False):
    """Eq. 7 root T[C,S] for every pair, to machine precision."""
    H = _f64(H)
    lam, dlam, c_abs, size = _f64(lam), _f64(dlam), _f64(c_abs), _f64(size)
    C, S = H.shape
    NL = lam.shape[0]
    assert c_abs.shape == (S, NL) and size.shape == (S,)
    T = np.empty((C, S), dtype=np.float64)
    it = np.empty((C, S), dtype=np.int32)
    lib().dust_ref_temperature(C, NL, S, _ptr(lam), _ptr(dlam), _ptr(c_abs),
                               _ptr(size), _ptr(H), _ptr(T), _ptr(it))
    return (T, it) if return_iters else T


def emission(T, lam, c_abs, weight, m_dust=None):
    """Eqs. 9-10: L[C,NL] = m[c] sum_s w_s C[s,l] B(lam_l, T[c,s])."""
    T = _f64(T)
    lam, c_abs, weight = _f64(lam), _f64(c_abs), _f64(weight)
    C, S = T.shape
    NL = lam.shape[0]
    md = _f64(m_dust) if m_dust is not None else None
    L = np.empty((C, NL), dtype=np.float64)
    lib().dust_ref_emission(C, NL, S, _ptr(lam), _ptr(c_abs), _ptr(weight),
                            _ptr(md), _ptr(T), _ptr(L))
    return L


def table_build(lam, dlam, c_abs, n_T=2000, t_min=3.0, t_max=1500.0):
    """Production variant (Sections 2 and 5): P[S, n_T], the grain power of
    Eq. 7 at n_T temperatures evenly spaced over [t_min, t_max]."""
    lam, dlam, c_abs = _f64(lam), _f64(dlam), _f64(c_abs)
    S, NL = c_abs.shape
    P = np.empty((S, n_T), dtype=np.float64)
    lib().dust_ref_table_build(NL, S, _ptr(lam), _ptr(dlam), _ptr(c_abs), int(n_T),
                               float(t_min), float(t_max), _ptr(P))
    return P


def table_temperature(H, P, t_min=3.0, t_max=1500.0):
    """T[C, S] by linear interpolation in the table P (see ``table_build``);
    returns (T, number of pairs outside the table, which get the end T)."""
    H, P = _f64(H), _f64(P)
    C, S = H.shape
    n_T = P.shape[1]
    assert P.shape == (S, n_T) and n_T >= 2
    T = np.empty((C, S), dtype=np.float64)
    n = lib().dust_ref_table_temperature(C, S, n_T, float(t_min), float(t_max), _ptr(P),
                                         _ptr(H), _ptr(T))
    return T, int(n)


def run(grid, J, m_dust=None, return_iters=False, Q=None, table=None):
    """The whole path on one grid: (H, T, L[, iters]).

    Q (optional, [C, S]) is heating from sources other than the radiation
    field, added to H before the balance is solved (Section 2: the heating
    need not be absorbed radiation); the returned H is the total.  ``table``
    = (n_T, t_min, t_max) selects the production variant of the temperature
    step (linear interpolation in a T table) instead of the exact root; iters
    are then zero."""
    H = heating(J, grid.c_abs, grid.dlam)
    if Q is not None:
        H = H + _f64(Q)
    if table is None:
        T, it = temperature(H, grid.lam, grid.dlam, grid.c_abs, grid.size, return_iters=True)
    else:
        n_T, t_min, t_max = table
        P = table_build(grid.lam, grid.dlam, grid.c_abs, n_T, t_min, t_max)
        T, _ = table_temperature(H, P, t_min, t_max)
        it = np.zeros(T.shape, dtype=np.int32)
    L = emission(T, grid.lam, grid.c_abs, grid.weight, m_dust)
    return (H, T, L, it) if return_iters else (H, T, L)


def reheat(grid, J0, m_dust, coupling, n_passes, Q=None, table=None):
    """Global iteration for dust that absorbs its own emission (Section 2):
    pass 0 heats with J0; pass n with J_n = J0 + coupling[c] * L_{n-1}[c, l],
    the stand-in for re-propagating the previous pass's emission.  Returns
    the list of (H, T, L) of every pass."""
    J0 = _f64(J0)
    g = _f64(coupling)[:, None]
    out = []
    J = J0
    for _ in range(n_passes):
        H, T, L = run(grid, J, m_dust, Q=Q, table=table)
        out.append((H, T, L))
        J = J0 + g * L
    return out


def fluct_distribution(J, grid, lev_T, lev_E):
    """Thermally fluctuating grains: P[C, S, M], the steady-state probability
    of each of a grain's M enthalpy levels (lev_E [S, M], J; at temperatures
    lev_T [S, M], K; level 0 the ground state E = T = 0) under single-photon
    heating by the field J[C, NL] and continuous cooling (see fluct_ref.c)."""
    J = _f64(J)
    lam, dlam, c_abs = _f64(grid.lam), _f64(grid.dlam), _f64(grid.c_abs)
    lev_T, lev_E = _f64(lev_T), _f64(lev_E)
    C, NL = J.shape
    S, M = lev_T.shape
    assert c_abs.shape == (S, NL) and lev_E.shape == (S, M) and M >= 2
    P = np.empty((C, S, M), dtype=np.float64)
    lib().dust_ref_fluct_distribution(C, NL, S, M, _ptr(lam), _ptr(dlam), _ptr(c_abs),
                                      _ptr(lev_T), _ptr(lev_E), _ptr(J), NL, _ptr(P))
    return P


def fluct_emission(P, grid, lev_T, m_dust=None):
    """L[C, NL] = m[c] sum_s w_s C[s,l] sum_j P[c,s,j] B(lam_l, T_sj)."""
    P = _f64(P)
    lam, c_abs, weight, lev_T = _f64(grid.lam), _f64(grid.c_abs), _f64(grid.weight), _f64(lev_T)
    C, S, M = P.shape
    NL = lam.shape[0]
    md = _f64(m_dust) if m_dust is not None else None
    L = np.empty((C, NL), dtype=np.float64)
    lib().dust_ref_fluct_emission(C, NL, S, M, _ptr(lam), _ptr(c_abs), _ptr(weight),
                                  _ptr(lev_T), _ptr(md), _ptr(P), _ptr(L))
    return L


def threads() -> int:
    return int(lib().dust_ref_get_threads())


def set_threads(n: int) -> None:
    lib().dust_ref_set_threads(int(n))
