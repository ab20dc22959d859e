"""Work and byte accounting for range-query scans.

Each stored value takes 4 bytes (float32 columns, Table 2 sizes are n * m * 4 bytes).
A single query reads only the columns it queries (vertical partitioning, section 5.5):
4 * N * k bytes, and writes 4 bytes per result identifier (or N / 8 bytes of bitmap).
"""

HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E, vendor figure
FP32_VALU_TFLOPS = 157.3    # MI355X vector fp32, vendor figure
CUS = 256
CLOCK_GHZ = 2.4
# Vector compares: 4 SIMDs x 16 lanes per CU retire one 32-bit compare per lane and clock
# (a wave64 instruction every 4 clocks per SIMD): 256 * 64 * 2.4e9 = 3.93e13 per second.
# The work of one row-predicate test is two compares, lo <= x and x <= hi (no single
# vector instruction decides a closed interval on this ISA: subtract then compare, or
# median-of-three then compare), so the shared scans' ALU roofline counts compares.
ALU_COMPARES_PEAK = CUS * 64 * CLOCK_GHZ * 1e9
COMPARES_PER_TEST = 2
# LDS: 128 bytes per clock per CU (32 banks of 4 bytes), the CDNA figure for wave-wide
# reads; 256 * 128 * 2.4e9 = 78.6 TB/s over the chip.
LDS_BYTES_PER_CLK = 128
LDS_PEAK_GBPS = CUS * LDS_BYTES_PER_CLK * CLOCK_GHZ
# Rank variant, per row and (group of up to 128 queries, column): one 4-byte bucket word
# and one row of query bitsets (4 words for a group of 128) read from LDS, plus the
# search probes inside the row's bucket (data-dependent, not counted).
RANK_LDS_BYTES_PER_LOOKUP = 4 + 16


def column_bytes(n_rows: int, n_dims: int) -> int:
    """Raw size of n_rows x n_dims float32 values."""
    return 4 * n_rows * n_dims


def query_bytes(n_rows: int, k: int, count: int, mode: str = "ids") -> int:
    """Algorithmic bytes of one single-query scan: every queried column read once, the
    result written once (ids: 4 B each; bitmap: one bit per row in 64-bit words), plus
    the 8-byte count."""
    out = {"ids": 4 * count, "bitmap": 8 * ((n_rows + 63) // 64), "count": 0}[mode]
    return column_bytes(n_rows, k) + out + 8
