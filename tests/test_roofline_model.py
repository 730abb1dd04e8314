"""Pin the byte accounting used for the roofline fraction to the bandwidth
model the paper prints (tests/golden/paper_bandwidth_model.txt)."""
import os

from paper_1301_4539_amd import roofline as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_bandwidth_model.txt")


def _rows():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        bw, vb, acc, mcs = line.split()[:4]
        yield float(bw), int(vb), float(acc), int(mcs)


def test_paper_bandwidth_model():
    rows = list(_rows())
    assert len(rows) == 7
    for bw, vb, acc, mcs in rows:
        # the paper prints the model rounded to whole MC/s (truncated in eq_ram_standard)
        v = R.cells_per_second(bw * 1e6, vb, acc) / 1e6
        assert abs(v - mcs) < 1.0, (bw, vb, acc, v, mcs)


def test_algorithmic_bytes():
    # two accesses per field (Sec. 3.2) plus a one-byte material index
    assert R.algorithmic_bytes(4) == 49 == R.bytes_per_cell_update(4, 2) + 1
    assert R.algorithmic_bytes(2) == 25
    assert abs(R.HBM_PEAK_GBPS * 1e9 / 49 / 1e9 - 163.27) < 0.01
