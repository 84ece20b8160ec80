"""The gather probe behind the measured gather ceilings: chained random reads
through a table, in global memory or staged in LDS, against the same chain
followed on the host."""
import numpy as np
import pytest

import synth
from tests._util import dev_u32, host_u32

pytestmark = pytest.mark.gpu
mbr = pytest.importorskip("paper_2203_04158_amd")


@pytest.mark.parametrize("entries,depth,lds,n", [(1 << 10, 1, False, 100003), (1 << 10, 3, True, 5000),
                                                 (1 << 14, 2, True, 77777), (1 << 20, 4, False, 1 << 20),
                                                 (1, 5, False, 33)])
def test_probe_gather_follows_the_chain(entries, depth, lds, n):
    mask = np.uint64(entries - 1)
    tab = synth.splitmix64(entries + depth, entries) & np.uint64(0xFFFFFFFF)
    idx = synth.splitmix64(n + 7, n) & np.uint64(0xFFFFFFFF)
    got = host_u32(mbr.probe_gather(dev_u32(tab), dev_u32(idx), depth=depth, lds=lds))
    i = idx & mask
    for _ in range(depth):
        i = tab[i.astype(np.int64)] & mask
    assert np.array_equal(got, i)


def test_probe_gather_rejects_bad_arguments():
    import torch
    t = torch.zeros(3, dtype=torch.int32, device="cuda")
    i = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(mbr.MbrError):
        mbr.probe_gather(t, i)                     # not a power of two
    big = torch.zeros(1 << 15, dtype=torch.int32, device="cuda")
    with pytest.raises(mbr.MbrError):
        mbr.probe_gather(big, i, lds=True)         # beyond 64 KB of LDS
    with pytest.raises(mbr.MbrError):
        mbr.probe_gather(big, i, depth=0)
