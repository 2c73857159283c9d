"""Parity at the benchmarked sizes, in the launch configuration bench.py
times (dataflow schedule, the default unit size and grid): one epoch from the
same state on the full Chung-Lu 1M graph (d = 128, sigmoid, FP32), the 2-D
random geometric 2M graph (d = 2, Student-t, FP32) and the SBM 4M graph in
the bf16 form (d = 128, Student-t, s = 10), each against the FP64 oracle on
every element: FP32 within 1e-5 relative (Frobenius) and every row within
1e-5 of its norm; bf16 against the oracle's bf16 emulation, >= 99.9% of the
bf16 images bit-identical and none more than one ulp apart."""
import time

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_helpers import assert_parity, bf16_compare, gpu_run, oracle_params, rel_fro

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def one_epoch(name, epoch_idx=1, emul=False):
    t0 = time.perf_counter()
    g, p = gg.workload(name)
    Z0 = gg.init_embedding(g.n, p["d"], p["z_seed"])
    print(f"{name}: n={g.n} nnz={g.nnz} generated in {time.perf_counter() - t0:.1f}s", flush=True)
    got = gpu_run(g, Z0, p, 1, first=epoch_idx)[0]
    t0 = time.perf_counter()
    ref = oracle.epoch(g, Z0, epoch_idx, oracle_params(p), emul=emul)
    print(f"{name}: oracle epoch {time.perf_counter() - t0:.1f}s", flush=True)
    return got, ref


@pytest.mark.parametrize("name", ["cl1m", "rgg2m"])
def test_fp32_one_epoch_full_size(name):
    got, ref = one_epoch(name)
    f, r = assert_parity(got, ref, 1e-5, 1e-5, name)
    print(f"{name}: relative Frobenius {f:.2e}, row-wise max {r:.2e}")


def test_bf16_one_epoch_full_size_sbm4m():
    got, ref = one_epoch("sbm4m", emul=True)
    same, ulps = bf16_compare(got, ref)
    err = rel_fro(got, ref)
    print(f"sbm4m bf16: images identical {same:.6f}, max ulp difference {ulps}, master rel err {err:.2e}")
    assert same >= 0.999 and ulps <= 1
    assert err <= 1e-4
