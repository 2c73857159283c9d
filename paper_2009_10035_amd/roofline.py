"""Algorithmic bytes of one update epoch (the unit of the roofline figures)."""


def algorithmic_bytes(n: int, nnz: int, d: int, b: int, s: int, precision: str) -> int:
    """HBM bytes one epoch must move: per stored edge its column index and the
    neighbour's row; per vertex its row pointer, batch lookups, own row read
    and new row written (plus the FP32 master in the bf16 form); per batch its
    negative rows once."""
    nb = (n + b - 1) // b
    if precision == "bf16":
        return nnz * (4 + 2 * d) + n * (10 * d + 12) + nb * s * 2 * d
    return nnz * (4 + 4 * d) + n * (8 * d + 12) + nb * s * 4 * d
