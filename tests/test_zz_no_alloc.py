"""The allocation-free entry point nnsort_sort_with_model_noalloc (static
device scratch) against nnsort_sort_with_model (caller workspace) through the
C ABI: the same output bits and the same round counts, on two calls in a row,
the second on a smaller input (the static array keeps the first call's
contents), for the FP32 and BF16 forms; and the oracle's sorted order."""
import ctypes

import numpy as np
import pytest

import oracle as O
import paper_1907_08817_amd as nn
from paper_1907_08817_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _noalloc(L, m, xd, sp):
    out = torch.empty_like(xd)
    st = nn.Stats()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.nnsort_sort_with_model_noalloc(ctypes.byref(m), ctypes.c_void_p(xd.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), xd.numel(), nn.F64, ctypes.byref(sp),
                                          ctypes.byref(st), stream)
    assert rc == 0, nn.STATUS.get(rc, rc)
    torch.cuda.synchronize()
    return out.cpu().numpy(), nn.stats_to_dict(st)


@pytest.mark.parametrize("form", [nn.FORM_FP32, nn.FORM_BF16])
def test_noalloc_matches_workspace_entry_point(form):
    L = nn._lib()
    for n, seed in ((1_552_000, 21), (300_001, 22)):
        print(f"noalloc form={form} n={n} seed={seed}", flush=True)
        x = W.gauss_mix(n, seed=seed)
        model = O.fit(x, H=64, sample_frac=0.01, steps=0)
        m = nn.model_from_dict(model)
        sp = nn.sort_params(form=form, stats_level=1)
        xd = torch.from_numpy(x).to(DEV)
        got, st = _noalloc(L, m, xd, sp)
        ref, rst = nn.nnsort_sort_with_model(m, xd, sp=sp)
        torch.cuda.synchronize()
        assert np.array_equal(got.view(np.uint64), ref.cpu().numpy().view(np.uint64))
        assert np.array_equal(got.view(np.uint64), O.sort_reference(x).view(np.uint64))
        for k in ("rounds", "collided", "placed", "residue", "unmapped", "big_bucket_keys", "fallback"):
            assert st[k] == rst[k], k


def test_noalloc_refuses_inputs_beyond_its_scratch():
    L = nn._lib()
    sp = nn.sort_params()
    m = nn.model_from_dict(O.fit(W.uniform(10_000), H=32, sample_frac=0.1, steps=0))
    xd = torch.zeros(1_552_001, dtype=torch.float64, device=DEV)
    out = torch.empty_like(xd)
    rc = L.nnsort_sort_with_model_noalloc(ctypes.byref(m), ctypes.c_void_p(xd.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), xd.numel(), nn.F64, ctypes.byref(sp),
                                          None, None)
    assert rc == -7
