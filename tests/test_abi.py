"""C-ABI checks that need no GPU: the library loads, exports every function
include/fpt.h declares, and its host-side validation rejects bad input with
the documented status codes."""

import ctypes
import math
import os
import re

import pytest

from paper_1802_05065_amd import _lib, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1802_05065_amd import build

        build.build()
    return _lib.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fpt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fpt_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(names) == bound


def test_version(lib):
    assert _lib.fpt_api_version() == 2


def test_plan_accepts_workloads_without_gpu(lib):
    for sets in ([workloads.plain_escape()], [workloads.switching_ramp()],
                 [workloads.uneven_overdamped()], workloads.batched_sets(16)):
        for prec in ("fp64", "fp32c"):
            h = _lib.fpt_plan(sets, prec)
            try:
                assert _lib.fpt_plan_workspace(h) > 0
            finally:
                _lib.fpt_plan_destroy(h)


@pytest.mark.parametrize("field,value,needle", [
    ("n_bins", 0, "n_bins"),
    ("n_bins", 4097, "n_bins"),
    ("dt", 0.0, "dt"),
    ("dt", math.inf, "dt"),
    ("T", -1.0, "T must"),
    ("max_steps", 0, "max_steps"),
    ("n_replicas", -5, "n_replicas"),
    ("model", 7, "model"),
    ("alpha", -0.1, "alpha"),
    ("threshold", math.inf, "threshold"),
    ("scheme", 2, "scheme"),
    ("rng", 2, "rng"),
])
def test_plan_rejects_bad_params(lib, field, value, needle):
    p = workloads.plain_escape()
    p[field] = value
    with pytest.raises(_lib.FptError) as e:
        _lib.fpt_plan([p], "fp64")
    assert e.value.status == _lib.FPT_E_INVAL
    assert needle in e.value.message


def test_overdamped_has_only_the_explicit_scheme(lib):
    p = workloads.uneven_overdamped(n_replicas=10)
    p["scheme"] = 1
    with pytest.raises(_lib.FptError) as e:
        _lib.fpt_plan([p], "fp64")
    assert "scheme" in e.value.message


def test_default_phi0_needs_bias_in_range(lib):
    p = workloads.plain_escape()
    p["phi0"] = math.nan
    p["gamma0"] = 1.5
    with pytest.raises(_lib.FptError) as e:
        _lib.fpt_plan([p], "fp64")
    assert "arcsin" in e.value.message


def test_plan_rejects_mixed_models_and_bad_tuning(lib):
    a = workloads.plain_escape()
    b = workloads.uneven_overdamped(n_replicas=10)
    with pytest.raises(_lib.FptError):
        _lib.fpt_plan([a, b], "fp64")
    for t in (dict(steps_per_launch=6), dict(replicas_per_lane=3), dict(waves_per_simd=9),
              dict(schedule=5)):
        with pytest.raises(_lib.FptError):
            _lib.fpt_plan([a], "fp64", t)
    with pytest.raises(_lib.FptError):
        _lib.fpt_plan([a], 7)


def test_histogram_before_simulate_is_a_state_error(lib):
    h = _lib.fpt_plan([workloads.plain_escape()], "fp64")
    try:
        with pytest.raises(_lib.FptError) as e:
            _lib.fpt_histogram(h, 0, 64)
        assert e.value.status == _lib.FPT_E_STATE
        with pytest.raises(_lib.FptError) as e:
            _lib.fpt_histogram_all(h, [64])
        assert e.value.status == _lib.FPT_E_STATE
    finally:
        _lib.fpt_plan_destroy(h)


def test_null_arguments(lib):
    import ctypes

    assert lib.fpt_plan(None, 1, 0, None, ctypes.byref(ctypes.c_void_p())) == _lib.FPT_E_INVAL
    assert lib.fpt_plan_workspace(None, None) == _lib.FPT_E_INVAL
    assert lib.fpt_simulate(None, None, None, None, None) == _lib.FPT_E_INVAL
    assert lib.fpt_histogram_all(None, None, None) == _lib.FPT_E_INVAL
    assert lib.fpt_server_create(None, 0, 0, 0, 0, None, None,
                                 ctypes.byref(ctypes.c_void_p())) == _lib.FPT_E_INVAL
    assert lib.fpt_simulate_noalloc(None, None, None, None) == _lib.FPT_E_INVAL
    assert lib.fpt_submit(None, None, None) == _lib.FPT_E_INVAL
    assert lib.fpt_poll(None, 1, None, None, None) == _lib.FPT_E_INVAL
    assert "NULL" in _lib.last_error()
    lib.fpt_plan_destroy(None)
    lib.fpt_server_destroy(None)


def test_workspace_grows_with_one_per_lane_schedule(lib):
    p = workloads.uneven_overdamped(n_replicas=2 ** 22)
    h1 = _lib.fpt_plan([p], "fp32c", dict(schedule=0))
    h2 = _lib.fpt_plan([p], "fp32c", dict(schedule=1))
    try:
        # one lane per replica: state for all 2^22 replicas
        assert _lib.fpt_plan_workspace(h2) >= 36 * 2 ** 22
        assert _lib.fpt_plan_workspace(h1) < _lib.fpt_plan_workspace(h2)
    finally:
        _lib.fpt_plan_destroy(h1)
        _lib.fpt_plan_destroy(h2)


def test_mt19937_plans(lib):
    p = dict(workloads.plain_escape(n_replicas=5000), rng=1)
    h = _lib.fpt_plan([p], "fp32c")
    h0 = _lib.fpt_plan([dict(p, rng=0)], "fp32c")
    try:
        # 624 words of generator state per slot, one slot per lane
        extra = _lib.fpt_plan_workspace(h) - _lib.fpt_plan_workspace(h0)
        assert extra >= 2496 * 256 * 4 * 8 * 64 // 2
    finally:
        _lib.fpt_plan_destroy(h)
        _lib.fpt_plan_destroy(h0)
    with pytest.raises(_lib.FptError) as e:
        _lib.fpt_plan([p, p], "fp64")
    assert "one parameter set" in e.value.message
    with pytest.raises(_lib.FptError) as e:
        _lib.fpt_plan([p], "fp64", dict(replicas_per_lane=2))
    assert "one replica per lane" in e.value.message


def test_plan_set_count_limit(lib):
    # histogram keys pack (set << 12 | bin) into 32 bits below the LDS tables'
    # empty marker 0xFFFFFFFF: 2^20 - 1 sets is the most a plan takes
    one = _lib.make_params(workloads.plain_escape(n_replicas=1))
    out = ctypes.c_void_p()
    arr = (_lib.FptParams * (1 << 20))(*([one] * (1 << 20)))
    st = lib.fpt_plan(arr, 1 << 20, _lib.FPT_FP64, None, ctypes.byref(out))
    assert st == _lib.FPT_E_INVAL
    assert b"parameter sets" in lib.fpt_last_error()
    st = lib.fpt_plan(arr, (1 << 20) - 1, _lib.FPT_FP64, None, ctypes.byref(out))
    assert st == _lib.FPT_OK
    lib.fpt_plan_destroy(out)


@pytest.mark.parametrize("model,gamma0,V0,ok", [
    (0, 1.0, 1.0, True), (0, 1.01, 1.0, False), (0, 0.9, 0.5, True),
    (1, 0.9, 0.5, False), (1, 1.5, 2.0, True), (1, 0.0, 0.0, False),
])
def test_default_start_needs_a_well(lib, model, gamma0, V0, ok):
    # NaN phi0 means the bottom of the well: arcsin(gamma0) (Eq. (10)) or
    # arcsin(gamma0 / V0) (overdamped), which must exist
    maker = workloads.plain_escape if model == 0 else workloads.uneven_overdamped
    p = dict(maker(n_replicas=4), gamma0=gamma0, V0=V0, phi0=math.nan, threshold=math.nan)
    if ok:
        _lib.fpt_plan_destroy(_lib.fpt_plan([p], "fp64"))
    else:
        with pytest.raises(_lib.FptError) as e:
            _lib.fpt_plan([p], "fp64")
        assert e.value.status == _lib.FPT_E_INVAL
        assert "default phi0" in e.value.message


@pytest.mark.parametrize("model,scheme", [(0, 2), (1, 1), (2, 0)])
def test_server_rejects_unknown_model_or_scheme(lib, model, scheme):
    # validated before the pool is touched (any aligned address will do)
    out = ctypes.c_void_p()
    st = lib.fpt_server_create(ctypes.c_void_p(256), 1 << 30, _lib.FPT_FP32C, model, scheme,
                               None, None, ctypes.byref(out))
    assert st == _lib.FPT_E_INVAL
    assert "model" in _lib.last_error() or "scheme" in _lib.last_error()


def test_header_is_pedantic_c99_and_cxx(tmp_path):
    # include/fpt.h is the boundary for C callers too: it compiles as strict
    # ISO C99 and as C++17 with every warning an error
    import subprocess

    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "use_fpt.c"
    src.write_text('#include <string.h>\n'
                   '#include "fpt.h"\n'
                   "int main(void) {\n"
                   "  fpt_params p;\n"
                   "  fpt_tuning t;\n"
                   "  fpt_moments m;\n"
                   "  memset(&p, 0, sizeof p);\n"
                   "  memset(&t, 0, sizeof t);\n"
                   "  memset(&m, 0, sizeof m);\n"
                   "  (void)p; (void)t; (void)m;\n"
                   "  return FPT_API_VERSION == 2 && FPT_NOALLOC_SCRATCH_BYTES > 0 ? 0 : 1;\n"
                   "}\n")
    for cmd in (["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                 "-fsyntax-only", "-I" + inc, str(src)],
                ["g++", "-std=c++17", "-pedantic", "-Wall", "-Wextra", "-Werror",
                 "-fsyntax-only", "-x", "c++", "-I" + inc, str(src)]):
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr


def test_missing_library_fails_loudly(monkeypatch):
    # no CPU fallback: without libfpt.so every entry point raises
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libfpt.so")
    with pytest.raises(RuntimeError, match="missing"):
        _lib.fpt_plan([workloads.plain_escape()], "fp64")
    with pytest.raises(RuntimeError, match="missing"):
        _lib.fpt_api_version()
    from paper_1802_05065_amd import api

    with pytest.raises(Exception):
        api.simulate(workloads.plain_escape(n_replicas=16), "fp64")
