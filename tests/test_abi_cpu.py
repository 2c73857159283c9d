"""The C ABI without a GPU: the library loads, exports every function the
header declares, the parameter struct matches the header's layout, and host
validation rejects bad parameters before any HIP call."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2009_10035_amd as f2v
from paper_2009_10035_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "f2v.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(f2v_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_function():
    lib = f2v.load()
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_binding.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", f2v._binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for name in names:
        assert re.search(r"\bT " + name + r"\b", out), name


def test_params_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "f2v.h"\n'
                   'int main(void){printf("%zu", sizeof(f2v_params));'
                   + "".join('printf(" %%zu", offsetof(f2v_params, %s));' % f for f, _ in f2v.Params._fields_)
                   + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(f2v.Params)
    assert vals[1:] == [getattr(f2v.Params, f).offset for f, _ in f2v.Params._fields_]


def good(**over):
    q = dict(n=1000, nnz=20000, d=128)
    q.update(over)
    n, nnz, d = q.pop("n"), q.pop("nnz"), q.pop("d")
    return f2v.make_params(n, nnz, d, **q)


def test_defaults_and_workspace():
    p = good()
    assert p.batch == 384 and p.s == 5 and abs(p.lr0 - 0.02) < 1e-9 and p.chunk == 0
    w128 = f2v.workspace_size(p)
    w256 = f2v.workspace_size(good(d=256))
    assert w256 > w128 > 1000 * 128 * 4
    assert f2v.workspace_size(good(precision="bf16")) < w128 * 2


def test_default_chunk_follows_graph_size():
    # chunk 0 picks 32 below 750k vertices and 64 from there on: the
    # workspace bound of chunk 0 equals that of the explicit choice
    for n, chunk in ((10_000, 32), (749_999, 32), (750_000, 64), (2_000_000, 64)):
        nnz = 20 * n
        auto = f2v.workspace_size(f2v.make_params(n, nnz, 128))
        assert auto == f2v.workspace_size(f2v.make_params(n, nnz, 128, chunk=chunk)), (n, chunk)
        other = 64 if chunk == 32 else 32
        assert auto != f2v.workspace_size(f2v.make_params(n, nnz, 128, chunk=other)), (n, other)


@pytest.mark.parametrize("field,value,status", [
    ("n", 0, "F2V_E_INVALID_ARG"), ("n", 2**29, "F2V_E_INVALID_ARG"), ("d", 0, "F2V_E_INVALID_ARG"),
    ("d", 1025, "F2V_E_INVALID_ARG"), ("d", 130, "F2V_E_UNSUPPORTED"), ("d", 65, "F2V_E_UNSUPPORTED"),
    ("batch", 0, "F2V_E_INVALID_ARG"), ("s", -1, "F2V_E_INVALID_ARG"), ("s", 65, "F2V_E_INVALID_ARG"),
    ("force", 5, "F2V_E_INVALID_ARG"), ("force", -1, "F2V_E_INVALID_ARG"), ("precision", 3, "F2V_E_INVALID_ARG"),
    ("lr0", 0.0, "F2V_E_INVALID_ARG"), ("walk_length", 65, "F2V_E_INVALID_ARG"), ("walk_length", -1, "F2V_E_INVALID_ARG"),
    ("fan_in", 3, "F2V_E_INVALID_ARG"), ("fan_in", 65, "F2V_E_INVALID_ARG"), ("late_window", 2**20 + 1, "F2V_E_INVALID_ARG"),
    ("lr0", float("nan"), "F2V_E_INVALID_ARG"), ("eps", 1.0, "F2V_E_INVALID_ARG"),
    ("eps", -0.1, "F2V_E_INVALID_ARG"), ("perm_mode", 2, "F2V_E_INVALID_ARG"),
    ("schedule", 4, "F2V_E_INVALID_ARG"), ("chunk", -1, "F2V_E_INVALID_ARG"), ("nnz", -1, "F2V_E_INVALID_ARG"),
    ("stage_negatives", 3, "F2V_E_INVALID_ARG"), ("stage_negatives", -1, "F2V_E_INVALID_ARG"),
])
def test_validation(field, value, status):
    p = good()
    setattr(p, field, value)
    with pytest.raises(f2v.F2VError) as ei:
        f2v.workspace_size(p)
    assert ei.value.name == status
    assert f2v.load().f2v_last_error(None)


def test_step_size_of_an_epoch():
    """eta_e of Algorithm 1: lr0 (constant) or lr0 (1 - e / E) (linear); an
    epoch at or past E under the linear schedule (eta <= 0) is refused, and
    f2v_epoch refuses it the same way."""
    lib = f2v.load()
    out = ctypes.c_float(0)
    p = good()
    assert lib.f2v_step_size(ctypes.byref(p), 7, ctypes.byref(out)) == 0 and out.value == pytest.approx(0.02)
    p = f2v.make_params(100, 200, 8, lr0=0.5, lr_schedule="linear", total_epochs=4)
    for e, want in ((0, 0.5), (1, 0.375), (3, 0.125)):
        assert lib.f2v_step_size(ctypes.byref(p), e, ctypes.byref(out)) == 0 and out.value == pytest.approx(want)
    for e in (4, 5, -1):
        assert _binding.STATUS[lib.f2v_step_size(ctypes.byref(p), e, ctypes.byref(out))] == "F2V_E_INVALID_ARG"


def test_linear_schedule_needs_epochs_and_bf16_needs_even_d():
    p = good(lr_schedule="linear")
    p.total_epochs = 0
    with pytest.raises(f2v.F2VError):
        f2v.workspace_size(p)
    with pytest.raises(f2v.F2VError) as ei:
        f2v.workspace_size(good(d=33, precision="bf16"))
    assert ei.value.name == "F2V_E_UNSUPPORTED"
    f2v.workspace_size(good(d=33))


def test_init_rejects_bad_pointers_without_touching_the_device():
    lib = f2v.load()
    p = good()
    ctx = ctypes.c_void_p()
    st = lib.f2v_init(ctypes.byref(p), None, None, None, None, 0, None, ctypes.byref(ctx))
    assert _binding.STATUS[st] == "F2V_E_INVALID_ARG"
    st = lib.f2v_init(ctypes.byref(p), 256, 512, 1024, 4096, 10, None, ctypes.byref(ctx))
    assert _binding.STATUS[st] == "F2V_E_OOM"
    st = lib.f2v_init(ctypes.byref(p), 256, 512, 1024, 4097, 1 << 40, None, ctypes.byref(ctx))
    assert _binding.STATUS[st] == "F2V_E_INVALID_ARG"   # misaligned workspace
    assert lib.f2v_epoch(None, 0) == 1 and lib.f2v_destroy(None) == 0
    assert lib.f2v_status_string(6) == b"device dependency wait timed out"


def test_static_workspace_entry_refuses_oversize_jobs_on_the_host():
    """f2v_train_static (callers that cannot allocate) refuses a job whose
    workspace exceeds its static array before any HIP call, and checks its
    arguments like f2v_init."""
    lib = f2v.load()
    lib.f2v_train_static.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    big = f2v.make_params(2_000_000, 40_000_000, 128)
    st = lib.f2v_train_static(ctypes.cast(ctypes.pointer(big), ctypes.c_void_p), 256, 512, 1024, 0, 1, None)
    assert _binding.STATUS[st] == "F2V_E_OOM"
    assert b"static workspace holds 268435456" in lib.f2v_last_error(None)
    p = good()
    st = lib.f2v_train_static(ctypes.cast(ctypes.pointer(p), ctypes.c_void_p), 256, 512, 1024, -1, 1, None)
    assert _binding.STATUS[st] == "F2V_E_INVALID_ARG"


def test_staged_negatives_limits():
    """The staged-negatives forms need the batch's rows to fit an LDS slot
    (s * d <= 2048 floats) and a schedule whose waves a workgroup shares (not
    the dynamic one); within that they are accepted."""
    ok = f2v.make_params(1000, 8000, 128, s=10, stage_negatives=1)
    assert f2v.workspace_size(ok) > 0
    for stage in (1, 2):
        with pytest.raises(f2v.F2VError) as ei:
            f2v.workspace_size(f2v.make_params(1000, 8000, 128, s=17, stage_negatives=stage))
        assert ei.value.name == "F2V_E_INVALID_ARG"
        with pytest.raises(f2v.F2VError) as ei:
            f2v.workspace_size(f2v.make_params(1000, 8000, 32, schedule="dynamic", stage_negatives=stage))
        assert ei.value.name == "F2V_E_UNSUPPORTED"
