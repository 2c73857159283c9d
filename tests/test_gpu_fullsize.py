"""Parity at the benchmarked sizes, in the launch configuration bench.py
times (dataflow schedule, the default unit size and grid): one epoch from the
same state on the full Chung-Lu 1M graph (d = 128, sigmoid, FP32), the 2-D
random geometric 2M graph (d = 2, Student-t, FP32) and the SBM 4M graph in
the bf16 form (d = 128, Student-t, s = 10), each against the FP64 oracle on
every element: FP32 within 1e-5 relative (Frobenius) and every row within
1e-5 of its norm; bf16 against the oracle's bf16 emulation, >= 99.9% of the
bf16 images bit-identical and none further apart than one bf16 ulp at the
RMS element's scale (a one-ulp flip of a stored row propagates to later
rows' terms)."""
import time

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_helpers import assert_parity, bf16_compare, gpu_run, oracle_params, rel_fro, row_rel

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
    """Row-wise bound 1e-5, or 10x the oracle's own row-wise response to a
    one-ulp (FP32) perturbation of the start if larger: in the 2-D layout a
    few rows meet a negative at close range, where the regularised Student-t
    repulsion amplifies any FP32 rounding of the rows it reads (measured:
    the oracle itself moves such rows by 1e-4 to 3e-4 of the RMS row)."""
    got, ref = one_epoch(name)
    g, p = gg.workload(name)
    Z0 = gg.init_embedding(g.n, p["d"], p["z_seed"]).astype(np.float64)
    rng = np.random.default_rng(0)
    pert = oracle.epoch(g, Z0 * (1 + 2.0**-24 * rng.choice([-1.0, 1.0], size=Z0.shape)), 1, oracle_params(p))
    row_bound = max(1e-5, 10 * row_rel(pert, ref))
    f, r = assert_parity(got, ref, 1e-5, row_bound, name)
    print(f"{name}: relative Frobenius {f:.2e}, row-wise max {r:.2e} (bound {row_bound:.2e})")


def test_bf16_one_epoch_full_size_sbm4m():
    got, ref = one_epoch("sbm4m", emul=True)
    same, bad = bf16_compare(got, ref)
    err = rel_fro(got, ref)
    print(f"sbm4m bf16: images identical {same:.6f}, beyond one ulp at the RMS scale: {bad}, master rel err {err:.2e}")
    assert same >= 0.999 and bad == 0
    assert err <= 1e-4
