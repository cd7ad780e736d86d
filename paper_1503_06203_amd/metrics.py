"""Operation and byte counts of the correlation, and MI355X peak figures.

Effective operations follow the paper's Eq. 2: a complex multiply-accumulate
is 8 operations (Sec. II-A), and only the N(N+1)/2 entries of the upper
triangle count, per channel and per time sample. Work done on redundant
entries below the diagonal, decode arithmetic and re-reads are never counted.
"""
from __future__ import annotations

OPS_PER_CMAC = 8                 # Sec. II-A
MAX_SAMPLES = 16_777_215         # |Re| <= 128 per sample keeps T*128 within int32

# MI355X (gfx950) published dense peaks and HBM bandwidth
PEAK_INT8_OPS = 5.0e15
PEAK_HBM_BYTES = 8.0e12


def vis_entries(n: int) -> int:
    return n * (n + 1) // 2


def effective_ops(n: int, f: int, t: int) -> int:
    """Eq. 2 per matrix, times channels and time samples."""
    return OPS_PER_CMAC * vis_entries(n) * f * t


def input_bytes(n: int, f: int, t: int) -> int:
    """One byte per (channel, sample, element): 4+4-bit packed input."""
    return n * f * t


def output_bytes(n: int, f: int) -> int:
    """int32 (re, im) per upper-triangle entry per channel."""
    return 8 * vis_entries(n) * f


def algorithmic_bytes(n: int, f: int, t: int, accumulate: bool) -> int:
    """Input read once, output written once (read and written if accumulating)."""
    return input_bytes(n, f, t) + output_bytes(n, f) * (2 if accumulate else 1)


def tile_count(n: int, tile: int) -> int:
    """Square tiles of edge ``tile`` covering the upper triangle (Fig. 1)."""
    nb = -(-n // tile)
    return nb * (nb + 1) // 2
