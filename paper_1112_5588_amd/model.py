"""Performance model of Sect. 2.2: code balance, execution time and the PCIe thresholds.

Byte counts used by the benchmark and the roofline report live here too, so that every
figure is computed one way.
"""
from __future__ import annotations


def code_balance_dp(alpha: float, n_nzr: float) -> float:
    """Eq. (1): bytes per flop of the ELLPACK/pJDS product in double precision: per non-zero
    8 B value + 4 B index + 8*alpha B of x, plus 16 B of y per row; 2 flops per non-zero."""
    return (8.0 + 4.0 + 8.0 * alpha + 16.0 / n_nzr) / 2.0


def t_mvm(n: float, n_nzr: float, alpha: float, b_gpu: float) -> float:
    """Eq. (2), device time of one product: (8N / B_GPU) [N_nzr (alpha + 3/2) + 2]."""
    return 8.0 * n / b_gpu * (n_nzr * (alpha + 1.5) + 2.0)


def t_pci(n: float, b_pci: float) -> float:
    """Eq. (2), host-link time for the right-hand side and the result: 16N / B_PCI."""
    return 16.0 * n / b_pci


def nnzr_bound_half_penalty(bw_ratio: float, alpha: float) -> float:
    """Eq. (3): T_MVM <= T_PCI (transfers cost at least half) for N_nzr at most this."""
    return 2.0 * (bw_ratio - 1.0) / (alpha + 1.5)


def nnzr_bound_tenth_penalty(bw_ratio: float, alpha: float) -> float:
    """Eq. (4): T_MVM >= 10 T_PCI (transfers cost under a tenth) for N_nzr at least this."""
    return (20.0 * bw_ratio - 2.0) / (alpha + 1.5)


def alg_bytes_spmv(nnz: int, n_rows: int, value_bytes: int = 8, index_bytes: int = 4) -> int:
    """Minimum traffic of y = A x: value and index per non-zero, x once and y once (the
    alpha = 1/N_nzr case of eq. (1) with y written, not read)."""
    return (value_bytes + index_bytes) * nnz + 2 * value_bytes * n_rows


def alg_bytes_spmmv(nnz: int, n_rows: int, k: int, value_bytes: int = 8) -> int:
    """Minimum traffic of Y = A X for k vectors: the matrix once, X and Y once each."""
    return (value_bytes + 4) * nnz + 2 * value_bytes * k * n_rows
