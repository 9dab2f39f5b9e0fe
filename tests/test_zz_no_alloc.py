"""rfi_flag_noalloc (the clip on the library's fixed device workspace)
against rfi_flag with a caller workspace, through the C ABI: two calls in a
row, the second on a smaller block, each bit for bit equal (mask, fit,
stream state), and sizes beyond the fixed workspace refused."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _stat(rng, n, frac):
    s = 0.075 + 0.002 * rng.standard_normal(n)
    k = int(frac * n)
    idx = rng.choice(n, size=k, replace=False)
    s[idx] += rng.uniform(0.003, 0.6, size=k)
    return np.clip(s, 1 / 19, 1.0)


def test_noalloc_matches_flag():
    import torch
    from paper_2512_16278_amd import rfi
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    L = rfi.lib()
    rng = np.random.default_rng(900)
    nstate = len(bytes(rfi.rfi_stream_state()))
    st_a = torch.zeros(nstate, dtype=torch.uint8, device=dev)
    st_b = torch.zeros(nstate, dtype=torch.uint8, device=dev)
    # the FAST block's cell count, then a smaller ragged block
    for nsub, nchan, frac in ((99, 4096, 0.03), (7, 333, 0.08)):
        n = nsub * nchan
        s = torch.from_numpy(_stat(rng, n, frac)).to(dev)
        status = torch.from_numpy((rng.uniform(size=n) < 0.001).astype(np.uint8)).to(dev)
        prot = torch.from_numpy((rng.uniform(size=nchan) < 0.02).astype(np.uint8)).to(dev)
        m_a = torch.full((n,), 7, dtype=torch.uint8, device=dev)
        m_b = torch.full((n,), 7, dtype=torch.uint8, device=dev)
        o_a = torch.zeros(48, dtype=torch.uint8, device=dev)
        o_b = torch.zeros(48, dtype=torch.uint8, device=dev)
        ws = rfi.flag_workspace(nsub, nchan, dev)
        say("noalloc: rfi_flag", nsub, nchan)
        rfi.rfi_flag(nsub, nchan, s, status, m_a, protect_chan=prot, state=st_a, out=o_a,
                     workspace=ws)
        torch.cuda.synchronize()
        say("noalloc: rfi_flag_noalloc", nsub, nchan)
        rfi.rfi_flag_noalloc(nsub, nchan, s, status, m_b, protect_chan=prot, state=st_b, out=o_b)
        torch.cuda.synchronize()
        assert torch.equal(m_a, m_b)
        assert (m_b <= 1).all()
        assert bytes(o_a.cpu().numpy()) == bytes(o_b.cpu().numpy())
        assert torch.equal(st_a, st_b)
        fs = rfi.flag_stats_from_bytes(o_b.cpu().numpy().tobytes())
        assert fs["iterations"] >= 1 and fs["nflag"] == int(m_b.sum())
    # beyond the fixed workspace: refused before any launch
    big = rfi.RFI_FLAG_NOALLOC_MAX_CELLS // 64 + 1
    code = L.rfi_flag_noalloc(big, 64, C.c_void_p(256), C.c_void_p(256), None, 3.0, 50, None,
                              C.c_void_p(256), None, None)
    assert code == rfi.RFI_E_INVALID
    assert b"fixed workspace" in L.rfi_last_error()
