"""Host logic of the measurement tools (no GPU): the gather probe's work
units cover every list entry exactly once, and the algorithmic bytes follow
their formula."""
import numpy as np

import graphgen as gg
from paper_2009_10035_amd.gather_ceiling import units_for
from paper_2009_10035_amd.roofline import algorithmic_bytes


def test_probe_units_cover_every_entry_once():
    g = gg.chung_lu(4000, 2.1, 20.0, 5)
    for chunk in (8, 32, 59):
        units, ubatch, nch = units_for(g.rowptr, g.n, chunk, 128, 1)
        cover = np.zeros(g.nnz, dtype=np.int64)
        for _, beg, ln, _ in units:
            cover[beg:beg + ln] += 1
        assert cover.min() == 1 and cover.max() == 1
        assert units[:, 2].max() <= chunk
        # one last unit per row (it takes the negatives), chunks numbered 0..nch-1
        last = units[units[:, 3] < 0]
        assert np.array_equal(np.sort(last[:, 0]), np.arange(g.n))
        assert np.array_equal(np.sort(units[units[:, 3] >= 0, 3]), np.arange(nch))
        # a row's units sit in its batch, the batches of a random order of the rows
        assert ubatch.min() == 0 and ubatch.max() == (g.n - 1) // 128


def test_algorithmic_bytes():
    n, nnz, d, b, s = 1000, 20000, 128, 384, 5
    nb = 3
    assert algorithmic_bytes(n, nnz, d, b, s, "fp32") == nnz * (4 + 4 * d) + n * (8 * d + 12) + nb * s * 4 * d
    assert algorithmic_bytes(n, nnz, d, b, s, "bf16") == nnz * (4 + 2 * d) + n * (10 * d + 12) + nb * s * 2 * d
    # the figure bench.py reports for the Chung-Lu workload
    assert algorithmic_bytes(1_000_000, 19_735_324, 128, 384, 5, "fp32") == 11_226_095_984
