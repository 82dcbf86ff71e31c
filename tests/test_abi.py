"""The C-ABI library loads, exports every declared entry point and rejects
bad arguments before touching the GPU (runs without one)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_0907_3768_amd as dust

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dust.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dust_[a-z_A-Z0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(dust.LIB_PATH):
        dust.build()
    return dust.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", dust.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (dust_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(L, n)


def test_version_and_no_error(L):
    assert b"gfx950" in L.dust_version()
    assert L.dust_last_error() == b""


def _desc(nl=8, s=2, lam=None, cabs=None, size=None):
    lam = np.geomspace(1e-7, 1e-3, nl) if lam is None else lam
    dl = np.full(nl, 1e-8)
    cabs = np.full((s, nl), 1e-14) if cabs is None else cabs
    w = np.ones(s)
    size = np.full(s, 1e-7) if size is None else size
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in (lam, dl, cabs, w, size)]
    d = dust.GridDesc(nl, s, *[a.ctypes.data for a in keep])
    return d, keep


@pytest.mark.parametrize("case,expect", [
    ("nl0", dust.DUST_EINVAL),
    ("s0", dust.DUST_EINVAL),
    ("s_big", dust.DUST_EUNSUPPORTED),
    ("lam_nonincreasing", dust.DUST_EINVAL),
    ("lam_negative", dust.DUST_EINVAL),
    ("cabs_negative", dust.DUST_EINVAL),
    ("cabs_nan", dust.DUST_EINVAL),
    ("size_zero", dust.DUST_EINVAL),
    ("bad_mode", dust.DUST_EINVAL),
    ("bad_mode3", dust.DUST_EINVAL),
    ("bad_ltab_linear", dust.DUST_EINVAL),
    ("bad_ltab", dust.DUST_EINVAL),
    ("bad_trange", dust.DUST_EINVAL),
    ("bad_fused_kernels", dust.DUST_EINVAL),
    ("options_reserved", dust.DUST_EINVAL),
    ("polish_plain", dust.DUST_EINVAL),
    ("polish_f32_lookup", dust.DUST_EINVAL),
    ("polish_table", dust.DUST_EINVAL),
])
def test_plan_create_rejects(L, case, expect):
    nl, s = 8, 2
    lam = np.geomspace(1e-7, 1e-3, nl)
    cabs = np.full((s, nl), 1e-14)
    size = np.full(s, 1e-7)
    opt = dust.Options(0, 0, 0.0, 0, 0, 0.0, 0.0, 0, 0, 0)
    if case == "nl0":
        nl = 0
    if case == "s0":
        s = 0
    if case == "s_big":
        s = 2048
        cabs = np.full((s, nl), 1e-14)
        size = np.full(s, 1e-7)
    if case == "lam_nonincreasing":
        lam = lam.copy(); lam[3] = lam[2]
    if case == "lam_negative":
        lam = lam.copy(); lam[0] = -1.0
    if case == "cabs_negative":
        cabs = cabs.copy(); cabs[1, 1] = -1e-14
    if case == "cabs_nan":
        cabs = cabs.copy(); cabs[0, 0] = np.nan
    if case == "size_zero":
        size = size.copy(); size[1] = 0.0
    if case == "bad_mode":
        opt.mode = 7
    if case == "bad_mode3":
        opt.mode = 3
    if case == "bad_ltab":
        opt.ltab_n = 3
    if case == "bad_ltab_linear":
        opt.mode, opt.ltab_n = dust.TABLE_LINEAR, 15
    if case == "bad_trange":
        opt.ltab_tmin, opt.ltab_tmax = 100.0, 50.0
    if case == "bad_fused_kernels":
        opt.fused_kernels = 3
    if case == "options_reserved":
        opt.reserved = 1
    if case == "polish_plain":           # the polish refines the mixed lookup only
        opt.newton_polish = 1
    if case == "polish_f32_lookup":
        opt.mode, opt.f32_lookup, opt.newton_polish = dust.MIXED, 1, 1
    if case == "polish_table":
        opt.mode, opt.newton_polish = dust.TABLE_LINEAR, 1
    d, keep = _desc(max(nl, 1), max(s, 1), lam if nl else None, cabs if s else None,
                    size if s else None)
    d.n_lambda, d.n_grains = nl, s
    h = ctypes.c_void_p()
    rc = L.dust_plan_create(ctypes.byref(d), ctypes.byref(opt), ctypes.byref(h))
    assert rc == expect
    assert h.value is None
    assert len(L.dust_last_error()) > 0


def test_null_arguments(L):
    d, keep = _desc()
    opt = dust.Options(0, 0, 0.0, 0, 0, 0.0, 0.0, 0, 0, 0)
    assert L.dust_plan_create(None, ctypes.byref(opt), ctypes.byref(ctypes.c_void_p())) == dust.DUST_EINVAL
    assert L.dust_plan_create(ctypes.byref(d), ctypes.byref(opt), None) == dust.DUST_EINVAL
    d.lambda_ = None
    assert L.dust_plan_create(ctypes.byref(d), ctypes.byref(opt), ctypes.byref(ctypes.c_void_p())) == dust.DUST_EINVAL
    assert L.dust_plan_destroy(None) == dust.DUST_OK
    nul = ctypes.c_void_p(0)
    assert L.dust_absorb(nul, 4, nul, 8, nul, 2, nul) == dust.DUST_EINVAL
    assert L.dust_solve_T(nul, 4, nul, 2, nul, 2, nul, nul) == dust.DUST_EINVAL
    assert L.dust_emit_sed(nul, 4, nul, 2, nul, nul, 8, nul) == dust.DUST_EINVAL
    assert L.dust_run_fused(nul, 4, nul, 8, nul, nul, 2, nul, 8, nul, nul) == dust.DUST_EINVAL
    x = dust.SolveExt(None, 0, 1, 0)
    assert L.dust_solve_T_ext(nul, 4, nul, 2, ctypes.byref(x), nul, 2, nul, nul) == dust.DUST_EINVAL
    assert L.dust_run_fused_ext(nul, 4, nul, 8, nul, ctypes.byref(x), nul, 2, nul, 8, nul,
                                nul) == dust.DUST_EINVAL
    assert L.dust_plan_prepare(nul, nul) == dust.DUST_EINVAL
    assert L.dust_plan_info(nul, nul, nul, nul) == dust.DUST_EINVAL
    assert L.dust_batch_launch(nul, nul) == dust.DUST_EINVAL
    assert L.dust_batch_info(nul, nul, nul) == dust.DUST_EINVAL
    assert L.dust_batch_destroy(nul) == dust.DUST_OK
    out = ctypes.c_void_p()
    assert L.dust_batch_create(nul, 0, nul, nul, nul, nul, nul, nul, nul, nul, nul, 0,
                               ctypes.byref(out)) == dust.DUST_EINVAL
    assert b"plan is NULL" in L.dust_last_error() or len(L.dust_last_error()) > 0


def test_product_package_has_no_oracle_dependency():
    """The product binding never imports the oracle (test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_0907_3768_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower(), f
                assert "dust_ref" not in src, f


def test_binding_constants_match_header():
    """The binding's mode values and counter layout follow include/dust.h."""
    text = open(os.path.join(ROOT, "include", "dust.h")).read()
    assert re.search(r"DUST_PLAIN_FP32 = 0", text) and re.search(r"DUST_MIXED = 1", text)
    assert re.search(r"DUST_TABLE_LINEAR = 2", text)
    assert (dust.PLAIN, dust.MIXED, dust.TABLE_LINEAR) == (0, 1, 2)
    body = re.search(r"typedef struct \{(.*?)\} dust_counters;", text, re.S).group(1)
    assert len(re.findall(r"int64_t\s+n_\w+;", body)) == dust.N_COUNTERS
    ext = re.search(r"typedef struct \{(.*?)\} dust_solve_ext;", text, re.S).group(1)
    assert ctypes.sizeof(dust.SolveExt) == 24 and "warm_start" in ext and "ldq" in ext


def test_probe_is_not_in_the_method_library():
    """The ALU throughput probes are measurement code: they live in their own
    library, which only the benchmark loads."""
    out = subprocess.run(["nm", "-D", "--defined-only", dust.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    assert "probe" not in out


@pytest.fixture(scope="module")
def P():
    from paper_0907_3768_amd import builder
    if not os.path.exists(builder.PROBE_LIB):
        dust.build()
    import bench
    return bench.probe_lib()


@pytest.mark.parametrize("kind,blocks,iters,null_out", [
    (0, 0, 16, False),         # no blocks
    (0, 1 << 21, 16, False),   # too many blocks
    (1, 4, 0, False),          # no iterations
    (2, 4, 16, True),          # NULL output
    (9, 4, 16, False),         # unknown kind
    (-1, 4, 16, False),
])
def test_probe_alu_rejects(P, kind, blocks, iters, null_out):
    """The ALU probe checks its arguments before any HIP call."""
    out = None if null_out else ctypes.c_void_p(16)  # never dereferenced: the call fails first
    assert P.alu_probe_run(kind, blocks, iters, out, None) == -1


def test_probe_constants_match_header():
    import bench
    text = open(os.path.join(ROOT, "paper_0907_3768_amd", "measure", "alu_probe.h")).read()
    for name, value in bench.PROBE_KINDS:
        key = {"exp2": "EXP2", "rcp": "RCP", "fma": "FMA", "exp2+fma": "EXP2_FMA",
               "term": "TERM", "fma64": "FMA64"}[name]
        assert re.search(rf"ALU_PROBE_{key} = {value}\b", text)


def test_batch_calls_reject_bad_arguments(L):
    """dust_batch_create and dust_batch_run check their arguments before any
    HIP call."""
    n = ctypes.c_void_p()
    nc = (ctypes.c_int64 * 1)(4)
    z = (ctypes.c_void_p * 1)(None)
    ld = (ctypes.c_int64 * 1)(8)
    args = [ctypes.cast(z, ctypes.c_void_p), 1, ctypes.cast(nc, ctypes.c_void_p)] + \
           [ctypes.cast(x, ctypes.c_void_p) for x in (z, ld, z, z, ld, z, ld)] + [None]
    assert L.dust_batch_run(*args, None) == dust.DUST_EINVAL       # plans[0] is NULL
    assert b"NULL" in L.dust_last_error()
    assert L.dust_batch_create(*args, 0, ctypes.byref(n)) == dust.DUST_EINVAL
    args[1] = 0
    assert L.dust_batch_run(*args, None) == dust.DUST_EINVAL       # no grids
    assert L.dust_batch_create(*args, 0, ctypes.byref(n)) == dust.DUST_EINVAL
    args[1] = 1
    args[10] = ctypes.c_void_p(12)                                  # misaligned counters
    assert L.dust_batch_run(*args, None) == dust.DUST_EINVAL
    assert L.dust_batch_create(*args, 9, ctypes.byref(n)) == dust.DUST_EINVAL  # bad flags
    assert L.dust_batch_form(None, None, None, None) == dust.DUST_EINVAL


def test_batch_run_noalloc_limits(L):
    """The no-allocation batched launch refuses, before any HIP call, more
    grids or more tiles than its fixed work-list array holds."""
    n = 257
    nc = (ctypes.c_int64 * n)(*([16] * n))
    z = (ctypes.c_void_p * n)()
    ld = (ctypes.c_int64 * n)(*([8] * n))
    v = lambda a: ctypes.cast(a, ctypes.c_void_p)
    args = [v(z), n, v(nc), v(z), v(ld), v(z), v(z), v(ld), v(z), v(ld), None, None]
    assert L.dust_batch_run_noalloc(*args) == dust.DUST_EINVAL
    assert b"256 grids" in L.dust_last_error()
    nc1 = (ctypes.c_int64 * 1)(16 * 600000)
    args = [v(z), 1, v(nc1), v(z), v(ld), v(z), v(z), v(ld), v(z), v(ld), None, None]
    assert L.dust_batch_run_noalloc(*args) == dust.DUST_EINVAL
    assert b"tiles" in L.dust_last_error()


def _levels(S, M, T=None, E=None):
    T = np.concatenate([[0.0], np.geomspace(3.0, 2000.0, M - 1)]) if T is None else T
    E = np.concatenate([[0.0], np.geomspace(1e-22, 1e-17, M - 1)]) if E is None else E
    keep = [np.ascontiguousarray(np.tile(x, (S, 1)), dtype=np.float64) for x in (T, E)]
    return dust.Levels(M, keep[0].ctypes.data, keep[1].ctypes.data), keep


@pytest.mark.parametrize("case", ["m1", "m_big", "t0", "e0", "e_flat", "t_nan", "null"])
def test_fluct_plan_rejects_bad_levels(L, case):
    """The fluctuating-grain plan checks its levels before any HIP call."""
    d, keep = _desc(nl=8, s=2)
    M = 6
    T = np.concatenate([[0.0], np.geomspace(3.0, 2000.0, M - 1)])
    E = np.concatenate([[0.0], np.geomspace(1e-22, 1e-17, M - 1)])
    if case == "m1":
        M, T, E = 1, T[:1], E[:1]
    if case == "m_big":
        M = 257
        T = np.concatenate([[0.0], np.geomspace(3.0, 2000.0, M - 1)])
        E = np.concatenate([[0.0], np.geomspace(1e-22, 1e-17, M - 1)])
    if case == "t0":
        T = T.copy(); T[0] = 1.0
    if case == "e0":
        E = E.copy(); E[0] = 1e-30
    if case == "e_flat":
        E = E.copy(); E[3] = E[2]
    if case == "t_nan":
        T = T.copy(); T[4] = np.nan
    lv, keep2 = _levels(2, M, T, E)
    if case == "null":
        lv.E = None
    h = ctypes.c_void_p()
    assert L.dust_fluct_plan_create(ctypes.byref(d), ctypes.byref(lv), ctypes.byref(h)) == \
        dust.DUST_EINVAL
    assert h.value is None and len(L.dust_last_error()) > 0


def test_fluct_calls_reject_null_plan(L):
    nul = ctypes.c_void_p(0)
    assert L.dust_fluct_solve_P(nul, 4, nul, 8, nul, 8, nul, nul) == dust.DUST_EINVAL
    assert L.dust_fluct_emit_sed(nul, 4, nul, 8, nul, nul, 8, 0, nul) == dust.DUST_EINVAL
    assert L.dust_fluct_plan_destroy(None) == dust.DUST_OK
