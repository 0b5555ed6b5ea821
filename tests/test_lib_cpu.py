"""CPU-side checks of libnnsort: it loads, exports every entry point that
include/nnsort.h declares, and its host-only paths (parameters, workspace
sizes, argument checks that return before any device work, model files)
behave as documented.  No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1907_08817_amd as nn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "nnsort.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nnsort_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = nn._lib()
    names = header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header_sizes():
    # sizes implied by the header's field lists (natural alignment, x86-64)
    assert ctypes.sizeof(nn.SortParams) == 32
    assert ctypes.sizeof(nn.FitParams) == 48
    assert ctypes.sizeof(nn.Model) == 8 + 16 + 4 * (64 * 4 + 64 * 64 + 1 + 3)
    assert ctypes.sizeof(nn.Stats) == 8 + 8 + 16 * 8 + 5 * 8 + 8 + 8 + 7 * 8


def test_default_params():
    sp, fp = nn.default_params()
    assert (sp.m, sp.eps, sp.tau, sp.form, sp.bf16_terms) == (1.25, 3, 1024, nn.FORM_FP32, 3)
    assert (fp.hidden, fp.batch, fp.steps, fp.init, fp.loss) == (32, 65536, 200, 1, 0)
    assert abs(fp.sample_frac - 0.01) < 1e-15


def test_workspace_size_grows_and_validates():
    sp, fp = nn.default_params()
    a = nn.workspace_size(10 ** 6, nn.F64, sp)
    b = nn.workspace_size(10 ** 7, nn.F64, sp)
    assert 0 < a < b
    assert nn.workspace_size(100, nn.F64, sp) > 0          # n <= tau: radix scratch only
    assert nn.workspace_size(10 ** 6, nn.F64, sp, fp) >= a
    bad = nn.sort_params(eps=0)
    with pytest.raises(nn.NNSortError):
        nn.workspace_size(10, nn.F64, bad)
    with pytest.raises(nn.NNSortError):
        nn.workspace_size(10, nn.F64, nn.sort_params(m=-1.0))
    with pytest.raises(nn.NNSortError):
        nn.workspace_size(10, nn.F64, nn.sort_params(form=7))
    with pytest.raises(nn.NNSortError):
        nn.workspace_size(2 ** 32, nn.F64, sp)               # beyond 32-bit indices
    with pytest.raises(nn.NNSortError):
        nn.workspace_size(10, nn.F64, sp, nn.fit_params(hidden=12))


def test_fit_sample_beyond_32_bit_offsets_rejected():
    # the sample is sorted with 32-bit offsets: 50 x 1e8 draws must be refused
    # (EINVAL) rather than planned; just below the limit is accepted
    sp, _ = nn.default_params()
    with pytest.raises(nn.NNSortError) as e:
        nn.workspace_size(10 ** 8, nn.F64, sp, nn.fit_params(sample_frac=50.0))
    assert e.value.status == -1
    assert nn.workspace_size(10 ** 8, nn.F64, sp, nn.fit_params(sample_frac=42.0)) > 0
    L = nn._lib()
    fp = nn.fit_params(sample_frac=50.0)
    m = nn.Model()
    p = ctypes.c_void_p(0x100000)
    assert L.nnsort_fit(p, 10 ** 8, 0, ctypes.byref(fp), ctypes.byref(m), p, 1 << 40, None) == -1


def test_argument_checks_before_device_work():
    L = nn._lib()
    sp, fp = nn.default_params()
    m = nn.Model()
    # null model / wrong version / width
    p = ctypes.c_void_p(0x100000)
    q = ctypes.c_void_p(0x900000)
    assert L.nnsort_sort_with_model(None, None, None, 0, 0, ctypes.byref(sp), None, 0, None, None) == -1
    assert L.nnsort_sort_with_model(ctypes.byref(m), p, q, 10, 0, ctypes.byref(sp), None, 0, None,
                                    None) == -4
    m.version, m.hidden = 1, 16
    # null pointers with n > 0
    assert L.nnsort_sort_with_model(ctypes.byref(m), None, None, 10, 0, ctypes.byref(sp), None, 0, None,
                                    None) == -1
    # overlapping input and output
    assert L.nnsort_sort_with_model(ctypes.byref(m), p, ctypes.c_void_p(0x100008), 10, 0, ctypes.byref(sp), None,
                                    0, None, None) == -1
    # workspace too small, or large enough but not 256-byte aligned (checked
    # before any launch)
    assert L.nnsort_sort_with_model(ctypes.byref(m), p, q, 5000, 0, ctypes.byref(sp), q, 16, None, None) == -2
    big = ctypes.c_size_t()
    assert L.nnsort_workspace_size(5000, 0, ctypes.byref(sp), None, ctypes.byref(big)) == 0
    assert L.nnsort_sort_with_model(ctypes.byref(m), p, q, 5000, 0, ctypes.byref(sp), ctypes.c_void_p(0x900008),
                                    big.value, None, None) == -2
    m64 = nn.Model()
    m64.version, m64.hidden = 1, 64
    assert L.nnsort_predict(ctypes.byref(m64), p, 10, 0, ctypes.byref(sp), None, None, ctypes.c_void_p(0x900008),
                            L.nnsort_model_device_bytes(), None) == -2
    assert "aligned" in L.nnsort_strerror(-2).decode()
    # fit: bad hidden width; workspace too small or not 256-byte aligned
    bad = nn.fit_params(hidden=5)
    assert L.nnsort_fit(p, 10, 0, ctypes.byref(bad), ctypes.byref(m), q, 1 << 20, None) == -1
    good = nn.fit_params(hidden=16)
    need = ctypes.c_size_t()
    assert L.nnsort_workspace_size(5000, 0, ctypes.byref(sp), ctypes.byref(good), ctypes.byref(need)) == 0
    assert L.nnsort_fit(p, 5000, 0, ctypes.byref(good), ctypes.byref(m), q, 64, None) == -2
    assert L.nnsort_fit(p, 5000, 0, ctypes.byref(good), ctypes.byref(m), ctypes.c_void_p(0x900008), need.value,
                        None) == -2
    assert L.nnsort_radix_sort(p, q, -1, 0, None, 0, None) == -1
    assert L.nnsort_mlp_forward(24, p, p, 4, p, None, None) == -1
    assert L.nnsort_adam_step(p, p, p, p, 4, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert "invalid" in L.nnsort_strerror(-1).decode()


def test_model_file_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    H = 24
    d = {"H": H, "lo": -3.5, "inv_range": 0.125,
         "theta": rng.standard_normal(H * H + 4 * H + 1).astype(np.float32)}
    m = nn.model_from_dict(d)
    path = str(tmp_path / "m.nnsm")
    nn.model_save(m, path)
    back = nn.model_to_dict(nn.model_load(path))
    assert back["H"] == H and back["lo"] == -3.5 and back["inv_range"] == 0.125
    assert np.array_equal(back["theta"], d["theta"])
    open(path, "r+b").write(b"XXXX")
    with pytest.raises(nn.NNSortError):
        nn.model_load(path)
    with pytest.raises(nn.NNSortError):
        nn.model_load(str(tmp_path / "missing"))


def test_parameter_names_are_checked():
    with pytest.raises(TypeError):
        nn.sort_params(epsilon=3)
    with pytest.raises(TypeError):
        nn.fit_params(delta=0.1)
    assert nn.fit_params(huber_delta=0.25).huber_delta == 0.25


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: asked for more it exits with a message
    before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("dtype", ["f64", "u64"])
def test_bench_host_parallel_sort_matches_numpy(dtype):
    """The benchmark's multi-threaded host sort (a context figure) returns
    numpy's sorted order, duplicates and ragged bucket sizes included."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    rng = np.random.default_rng(7)
    if dtype == "f64":
        x = np.concatenate([rng.lognormal(0.0, 2.0, 200_003), np.full(5000, 3.25), rng.random(1001)])
    else:
        x = np.concatenate([rng.zipf(1.3, 200_003).astype(np.uint64), np.arange(999, dtype=np.uint64)])
    rng.shuffle(x)
    for threads in (1, 3, 8):
        assert np.array_equal(bench.host_parallel_sort(x, threads), np.sort(x))


def test_noalloc_size_check_precedes_device_work():
    # beyond the 64 MiB static scratch: ETOOBIG from the host-side check,
    # before anything touches a device (this container has none)
    L = nn._lib()
    sp, _ = nn.default_params()
    m = nn.Model()
    m.version, m.hidden = 1, 32
    p, q = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x90000000)
    assert L.nnsort_sort_with_model_noalloc(ctypes.byref(m), p, q, 10 ** 7, 0, ctypes.byref(sp), None, None) == -7
    assert L.nnsort_sort_with_model_noalloc(None, p, q, 10, 0, ctypes.byref(sp), None, None) == -1
    assert nn.workspace_size(1_552_000, nn.F64, sp) <= 64 << 20 < nn.workspace_size(1_552_001, nn.F64, sp)
