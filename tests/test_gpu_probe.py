"""The plain HBM streams behind the bench's ceilings: the copy is exact, the
fill writes its pattern everywhere and nowhere else, the read changes
neither its source nor more than the 16-byte sink of its destination.
Sizes are ragged against the grid-stride unrolling (four words per lane)."""
import pytest
import torch

import paper_2604_16590_amd as la
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (64 << 20) + 16 * 13])
def test_copy_is_exact(nbytes):
    dev = require_gpu()
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device=dev)
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device=dev)
    la.stream_probe("copy", dst[:nbytes], src)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].count_nonzero()) == 0


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (64 << 20) + 16 * 13])
def test_write_fills_the_pattern_only_in_range(nbytes):
    dev = require_gpu()
    buf = torch.zeros((nbytes + 64) // 4, dtype=torch.int32, device=dev)
    la.stream_probe("write", buf[:nbytes // 4], pattern=0x5A5AA5A5)
    torch.cuda.synchronize()
    want = torch.tensor(0x5A5AA5A5, dtype=torch.int64).to(torch.int32).item()
    assert bool((buf[:nbytes // 4] == want).all())
    assert int(buf[nbytes // 4:].count_nonzero()) == 0


def test_read_leaves_source_and_sink_tail_unchanged():
    dev = require_gpu()
    nbytes = (32 << 20) + 16 * 7
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device=dev)
    keep = src.clone()
    sink = torch.full((64,), 7, dtype=torch.uint8, device=dev)
    la.stream_probe("read", sink, src)
    torch.cuda.synchronize()
    assert torch.equal(src, keep)
    assert bool((sink[16:] == 7).all())
