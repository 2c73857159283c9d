"""The entry point for callers that cannot allocate (f2v_train_static): its
workspace is the library's static device array.  Its result equals the
allocating path's (f2v_init with a caller workspace, the same epochs,
f2v_sync_embedding) bit for bit, on two calls in a row, the second with a
smaller job; a job too large for the array is refused before device work."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_2009_10035_amd as f2v
from gpu_helpers import device_graph, gpu_run, lib_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def static_run(g, Z0, p, first, epochs):
    lib = f2v.load()
    lib.f2v_train_static.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    rowptr, colidx = device_graph(g)
    z = torch.from_numpy(np.ascontiguousarray(Z0, dtype=np.float32)).cuda()
    params = lib_params(g, p)
    st = lib.f2v_train_static(ctypes.cast(ctypes.pointer(params), ctypes.c_void_p), rowptr.data_ptr(),
                              colidx.data_ptr(), z.data_ptr(), first, epochs,
                              torch.cuda.current_stream().cuda_stream)
    return st, z.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_static_workspace_equals_allocating_path(precision):
    big = gg.chung_lu(60000, 2.1, 16.0, 1)
    small = gg.erdos_renyi(5000, 10.0, 2)
    for g, d, first, epochs in ((big, 128, 0, 3), (small, 32, 2, 2)):
        p = dict(d=d, batch=384, s=5, force="sigmoid", lr0=0.02, seed=7, precision=precision)
        Z0 = gg.init_embedding(g.n, d, 3)
        st, got = static_run(g, Z0, p, first, epochs)
        assert st == 0, f2v.load().f2v_last_error(None)
        ref = gpu_run(g, Z0, p, epochs, first=first, snapshots=False)[-1]
        assert np.array_equal(got, ref), (g.n, precision)


def test_static_workspace_refuses_a_job_too_large():
    lib = f2v.load()
    p = f2v.make_params(2_000_000, 40_000_000, 128)
    lib.f2v_train_static.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    st = lib.f2v_train_static(ctypes.cast(ctypes.pointer(p), ctypes.c_void_p), 256, 512, 1024, 0, 1, None)
    assert f2v._binding.STATUS[st] == "F2V_E_OOM"
    assert b"static workspace holds 268435456" in lib.f2v_last_error(None)
