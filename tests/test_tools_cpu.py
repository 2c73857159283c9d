"""Host logic of the measurement (no GPU): the algorithmic bytes follow
their formula."""
from paper_2009_10035_amd.roofline import algorithmic_bytes


def test_algorithmic_bytes():
    n, nnz, d, b, s = 1000, 20000, 128, 384, 5
    nb = 3
    assert algorithmic_bytes(n, nnz, d, b, s, "fp32") == nnz * (4 + 4 * d) + n * (8 * d + 12) + nb * s * 4 * d
    assert algorithmic_bytes(n, nnz, d, b, s, "bf16") == nnz * (4 + 2 * d) + n * (10 * d + 12) + nb * s * 2 * d
    # the figure bench.py reports for the Chung-Lu workload
    assert algorithmic_bytes(1_000_000, 19_735_324, 128, 384, 5, "fp32") == 11_226_095_984
