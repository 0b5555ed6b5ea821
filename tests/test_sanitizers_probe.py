"""Host paths of libnnsort that the sanitizer build should walk and that need
no GPU: the BF16 operand preparation of nnsort_predict (it runs before the
first device call, which then fails without a device), and parameter checks
over a grid of sizes.  Runs in the plain CPU suite too."""
import ctypes
import math

import numpy as np
import pytest

import paper_1907_08817_amd as nn

try:
    import torch
    _HAS_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    _HAS_GPU = False


def _models():
    rng = np.random.default_rng(4)
    out = []
    for H in (8, 32, 64):
        th = rng.standard_normal(H * H + 4 * H + 1).astype(np.float32)
        th[:H] *= 1e6                                   # steep layer-1 units
        out.append({"H": H, "lo": -3.0, "inv_range": 0.25, "theta": th})
    th = out[-1]["theta"].copy()
    th[2 * 64 + 5] = 1e-38                              # a W2 entry that cannot be scaled exactly
    out.append({"H": 64, "lo": 0.0, "inv_range": 1.0, "theta": th})
    th = out[-1]["theta"].copy()
    th[7] = np.nan                                      # non-finite: maps no key
    out.append({"H": 64, "lo": 0.0, "inv_range": 1.0, "theta": th})
    return out


@pytest.mark.skipif(_HAS_GPU, reason="walks the host path up to the first device call, which needs no GPU here")
def test_predict_host_path_without_device():
    L = nn._lib()
    sp = nn.sort_params(form=nn.FORM_BF16)
    need = L.nnsort_model_device_bytes()
    p = ctypes.c_void_p(0x7f0000000000)
    for d in _models():
        m = nn.model_from_dict(d)
        rc = L.nnsort_predict(ctypes.byref(m), p, 1000, nn.F64, ctypes.byref(sp), p, p, p, need, None)
        assert rc == -3  # EHIP: the host work is done, the device copy fails


def test_workspace_sizes_over_a_grid():
    sp, fp = nn.default_params()
    last = 0
    for e in range(0, 31, 3):
        n = 2 ** e + 17
        for m in (1.0, 1.25, 2.0):
            b = nn.workspace_size(n, nn.F64, nn.sort_params(m=m), fp)
            assert b > 0 and b % 256 == 0
        b = nn.workspace_size(n, nn.U64, sp)
        assert b >= last
        last = b
    for frac in (1e-6, 0.01, 1.0, 30.0):
        assert nn.workspace_size(10 ** 6, nn.F64, sp, nn.fit_params(sample_frac=frac)) > 0
    assert math.isfinite(float(last))
