"""The random-read probe (skis_probe_random_read), the measurement aid behind the
random-access ceiling: every row size reads the table it is given, in bounds, and bad
arguments are refused."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

MARK = np.int32(np.uint32(0x9E3779B9).view(np.int32))  # the fold value that makes the probe store


@pytest.fixture(scope="module")
def skis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03565_amd import skis as s
    s.lib()
    return s


@pytest.mark.parametrize("row_bytes", [8, 16, 32, 64, 128])
def test_probe_reads_the_rows(skis, row_bytes):
    print("[gpu-probe] row_bytes", row_bytes, flush=True)
    rows = 1 << 14
    # every row folds (xor of its 32-bit words) to MARK: its first word MARK, the rest zero
    t = torch.zeros(rows * row_bytes // 4, dtype=torch.int32, device="cuda")
    t[:: row_bytes // 4] = int(MARK)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    # one read per thread of the probe's grid (16 workgroups of 256 per compute unit): each
    # thread's fold is MARK, so the probe stores it
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    skis.probe_random_read(t, row_bytes, cus * 16 * 256, sink)
    torch.cuda.synchronize()
    assert int(sink.item()) == int(MARK)
    # a zero table folds to 0: nothing is stored, whatever the number of reads
    z = torch.zeros(rows * row_bytes // 4, dtype=torch.int32, device="cuda")
    sink.zero_()
    for reads in (0, 1, 1000, 3 * cus * 16 * 256 + 17):
        skis.probe_random_read(z, row_bytes, reads, sink)
    torch.cuda.synchronize()
    assert int(sink.item()) == 0


def test_probe_refuses_bad_arguments(skis):
    t = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    for rb in (0, 4, 12, 256):
        with pytest.raises(skis.SkisError):
            skis.probe_random_read(t, rb, 10, sink)
    with pytest.raises(skis.SkisError):  # fewer bytes than one row: no rows
        skis.probe_random_read(t[:4], 8, 10, sink)
    with pytest.raises(skis.SkisError):  # not 16-byte aligned
        skis.probe_random_read(t[1:1025], 8, 10, sink)
    with pytest.raises(skis.SkisError):  # 2^32 reads or more
        skis.probe_random_read(t, 8, 1 << 32, sink)
    torch.cuda.synchronize()
    assert int(sink.item()) == 0
