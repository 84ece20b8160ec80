"""The allocation-free gradient entry point (mbr_mlp_gradients_noalloc)
against the allocating one (mbr_mlp_gradients), through the C ABI: the same
kernels over a static scratch array, so the gradients and the loss must be
bitwise equal; two calls in a row, the second with a smaller batch, so the
second runs on scratch the first left behind.  Both are also held to the
fp64 oracle's bound of the gradient test."""
import numpy as np
import pytest

from oracle import mlp as OM
import synth
from tests._util import dev_u32, say

pytestmark = pytest.mark.gpu
mbr = pytest.importorskip("paper_2203_04158_amd")
torch = pytest.importorskip("torch")


def _params(seed):
    u = 2 * synth.uniform01(seed, 6337) - 1
    u[:2048] *= 0.4
    u[2112:6208] *= 0.25
    u[2048:2112] *= 0.1
    u[6208:6272] *= 0.1
    u[6272:6336] *= 0.3
    return u.astype(np.float32)


def _bf16(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _split(flat):
    f = np.asarray(flat, dtype=np.float64)
    return [f[0:2048].reshape(64, 32), f[2048:2112], f[2112:6208].reshape(64, 64),
            f[6208:6272], f[6272:6336], float(f[6336])]


def test_noalloc_gradients_match_allocating_entry_point():
    grad = torch.empty(6337, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for call, (B, seed) in enumerate(((8192, 21), (320, 22))):
        say("no-alloc gradients: call", call, "B", B)
        p32 = _params(seed)
        q = synth.splitmix64(seed + 1, B) & np.uint64(0xFFFFFFFF)
        tgt = synth.uniform01(seed + 2, B).astype(np.float32)
        pd, qd, td = torch.from_numpy(p32).cuda(), dev_u32(q), torch.from_numpy(tgt).cuda()
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        mbr.mlp_gradients_noalloc(pd, qd, td, grad, loss)
        torch.cuda.synchronize()
        g_ref, l_ref = mbr.mlp_gradients(pd, qd, td)
        assert torch.equal(grad, g_ref), (grad - g_ref).abs().max()
        assert torch.equal(loss, l_ref)
        # the oracle's bar (fp32 accumulation over the batch)
        P = _split(_bf16(p32))
        G = OM.gradients(P, OM.features(q), tgt.astype(np.float64))
        for a, b in zip(_split(grad.cpu().numpy()), G):
            a, b = np.atleast_1d(a), np.atleast_1d(b)
            assert np.abs(a - b).max() <= 1e-4 * max(1e-12, np.abs(b).max())


def test_noalloc_gradients_reject_oversized_batch():
    p = torch.zeros(6337, dtype=torch.float32, device="cuda")
    q = torch.zeros(8256, dtype=torch.int32, device="cuda")
    t = torch.zeros(8256, dtype=torch.float32, device="cuda")
    g = torch.empty(6337, dtype=torch.float32, device="cuda")
    l = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(mbr.MbrError) as ei:
        mbr.mlp_gradients_noalloc(p, q, t, g, l)
    assert ei.value.status == -6 and "static scratch" in str(ei.value)
    with pytest.raises(mbr.MbrError):
        mbr.mlp_gradients_noalloc(p, q[:100], t[:100], g, l)   # not a multiple of 64
