"""Byte accounting of the Yee update (the paper's bandwidth model).

A Yee cell holds six field values.  If every field update costs `accesses`
memory accesses of `value_bytes` each, one cell-update moves
value_bytes * 6 * accesses bytes and a memory system of bandwidth B sustains
B / (value_bytes * 6 * accesses) cell-updates per second (Sec. 2.2 for six
accesses per field, Sec. 3.1 three, Sec. 3.2 two, Sec. 3.4 one).

The algorithmic traffic used for the roofline fraction is the interleaved
count of Sec. 3.2 -- each component read once and written once, no temporal
reuse -- plus the one-byte material index of this library:
    B_alg = 2 * 6 * value_bytes + 1  bytes per cell-update
(49 B in FP32, 25 B with FP16/BF16 storage).
"""

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published peak


def bytes_per_cell_update(value_bytes: int, accesses_per_field: float) -> float:
    return value_bytes * 6 * accesses_per_field


def cells_per_second(bandwidth_bytes_s: float, value_bytes: int, accesses_per_field: float) -> float:
    return bandwidth_bytes_s / bytes_per_cell_update(value_bytes, accesses_per_field)


def algorithmic_bytes(value_bytes: int, material_index: bool = True) -> int:
    return 2 * 6 * value_bytes + (1 if material_index else 0)
