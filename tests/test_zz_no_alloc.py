"""GPU test of ipb_complete_static, the entry point for callers that cannot
allocate: through the C ABI, its output equals ipb_complete_ws's bit for bit
on two calls in a row, the second with a smaller frame (the static array
keeps the first call's contents, which must not leak into the second)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1802_00036_amd import _lib as L
from paper_1802_00036_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _bits(t):
    return np.ascontiguousarray(t.cpu().numpy()).view(np.uint32)


def _with_ws(x, cp):
    H, W = x.shape
    lib = L.lib()
    nb = int(lib.ipb_workspace_bytes(H, W, ctypes.byref(cp)))
    ws = api._workspace(nb, x.device)
    out = torch.full_like(x, -7.0)
    h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.check(lib.ipb_complete_ws(ctypes.c_void_p(x.data_ptr()), H, W, ctypes.byref(cp), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(ws.data_ptr()), nb, h), "ipb_complete_ws")
    torch.cuda.synchronize()
    return out


def _static(x, cp):
    H, W = x.shape
    out = torch.full_like(x, -7.0)
    torch.cuda.synchronize()
    h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.check(L.lib().ipb_complete_static(ctypes.c_void_p(x.data_ptr()), H, W, ctypes.byref(cp),
                                        ctypes.c_void_p(out.data_ptr()), h), "ipb_complete_static")
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("params", ["default", "offset140"])
def test_static_scratch_equals_workspace_call(params):
    p = api.Params(max_depth=140.0) if params == "offset140" else api.Params()
    cp = p.to_c()
    big = torch.from_numpy(synth.lidar_frame(375, 1242, seed=[40, 0], n_rows=64, density=0.05).sparse).to(DEV)
    small = torch.from_numpy(synth.lidar_frame(130, 333, seed=[40, 1], n_rows=40, density=0.08).sparse).to(DEV)
    for name, x in (("375x1242", big), ("130x333 after 375x1242", small)):
        print(f"[static scratch] {params} {name}", flush=True)
        got = _static(x, cp)
        want = _with_ws(x, cp)
        assert np.array_equal(_bits(got), _bits(want)), name


def test_static_scratch_largest_serving_frame_and_refusal():
    cp = api.Params(max_depth=140.0).to_c()
    x = torch.from_numpy(synth.lidar_frame(1024, 4096, seed=[40, 2], n_rows=128, density=0.03).sparse).to(DEV)
    print("[static scratch] 1024x4096", flush=True)
    assert np.array_equal(_bits(_static(x, cp)), _bits(_with_ws(x, cp)))
    y = torch.zeros((4096, 4096), dtype=torch.float32, device=DEV)
    out = torch.empty_like(y)
    st = L.lib().ipb_complete_static(ctypes.c_void_p(y.data_ptr()), 4096, 4096, ctypes.byref(cp),
                                     ctypes.c_void_p(out.data_ptr()), None)
    assert st == L.IPB_ERR_SCRATCH
