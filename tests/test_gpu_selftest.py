"""The publication protocol across XCDs (f2v_selftest_publish, through the C
ABI): writer and reader waves on different XCDs exchange rows exactly as the
update kernel's units do (device-scope row stores, a wait for their
completion, a device-scope flag store; flag polls and device-scope row
loads).  No word may be read stale and no poll may run into the wait bound,
also with four self-tests running at once on separate streams (as the
serving form's jobs do)."""
import pytest
import torch

import paper_2009_10035_amd as f2v

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_publication_is_never_read_stale():
    r = f2v.selftest_publish(pairs=512, rounds=20000)
    assert r == {"stale": 0, "timeouts": 0, "completed": 512}, r


def test_publication_on_concurrent_streams():
    streams = [torch.cuda.Stream() for _ in range(4)]
    out = [None] * 4
    for i, s in enumerate(streams):
        with torch.cuda.stream(s):
            out[i] = f2v.selftest_publish(pairs=64, rounds=20000)
    torch.cuda.synchronize()
    assert all(o == {"stale": 0, "timeouts": 0, "completed": 64} for o in out), out


def test_selftest_rejects_bad_arguments():
    lib = f2v.load()
    out = (__import__("ctypes").c_uint32 * 3)()
    assert f2v._binding.STATUS[lib.f2v_selftest_publish(0, 10, None, 0, out, None)] == "F2V_E_INVALID_ARG"
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    st = lib.f2v_selftest_publish(8, 10, ws.data_ptr(), ws.numel(), out, None)
    assert f2v._binding.STATUS[st] == "F2V_E_INVALID_ARG"   # buffer too small
