"""GPU: long sub-intervals (Table 1 runs 0.05 - 10 s sub-intervals; 10 s of
49.152 us samples is L = 203,450), above the int32 bound of the sums.

* rfi_ccm_accumulate_long: int64 sums bit-exact against the oracle at
  L = 40,960 and 203,450, with saturated stretches that drive S_aa past 2^31,
  for several beam classes, a sample offset and a ragged channel count.
* rfi_eig_batched_long: the FP64 tridiagonal solver on those sums, statistic
  within 1e-12 of the oracle, eigenvalues within 1e-6 of lambda_1.
* rfi_process_block at L = 203,450 equals the separate long calls bit for bit
  and its mask the oracle clip of the same statistic.
The full FAST-shaped 10 s sub-interval is checked in test_gpu_fullsize.py.
"""
import numpy as np
import pytest

from gpu_util import say, upload
from oracle import ccm, clip, pipeline

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_16278_amd import rfi
    rfi.lib()
    return torch.device("cuda:0")


def _data(nbeam, nsamp, nchan, seed):
    rng = np.random.default_rng(seed)
    x = 128 + 25 * rng.standard_normal((nbeam, nsamp, nchan))
    t = np.arange(nsamp)
    g = rng.uniform(0.3, 2.0, nbeam)
    x[:, :, 1] += 8 * g[:, None] * np.sin(2 * np.pi * t / 97.0)[None, :]   # common mode
    x = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    x[0, :34000, 0] = 255                    # S_00 of cell (0, 0) beyond 2^31
    x[1, 5:34100:2, 2] = 0                   # large alternating variance
    x[1, 6:34100:2, 2] = 255
    return x


def _long_sums(dev, x, L, nsub, t0, nchan):
    import torch
    from paper_2512_16278_amd import rfi
    nb = x.shape[0]
    buf = upload(x, dev)
    blk = rfi.make_block(buf, nchan)
    nrow = nb + nb * (nb + 1) // 2
    sums = torch.full((nsub * nchan, nrow), -7, dtype=torch.int64, device=dev)
    cnt = torch.full((nsub,), -7, dtype=torch.int32, device=dev)
    ws = torch.empty(rfi.rfi_ccm_long_workspace_size(nb, nchan, nsub), dtype=torch.uint8,
                     device=dev)
    say("long sums", nb, nchan, L, nsub, t0)
    rfi.rfi_ccm_accumulate_long(blk, t0, L, nsub, sums, cnt, ws)
    torch.cuda.synchronize()
    return buf, blk, sums, cnt


def _packed(S, S2):
    nsub, nchan, nb = S.shape
    iu = np.triu_indices(nb)
    rec = np.concatenate([S.reshape(-1, nb), S2.reshape(-1, nb, nb)[:, iu[0], iu[1]]], axis=1)
    return rec


@pytest.mark.parametrize("nb,nchan,L,nsub,t0", [
    (3, 5, 40960, 2, 3), (19, 33, 40960, 1, 0), (19, 7, 203450, 1, 17), (36, 17, 66051, 2, 1),
    (72, 3, 203450, 1, 0), (2, 64, 33026, 3, 0)])
def test_long_sums_bit_exact(dev, nb, nchan, L, nsub, t0):
    x = _data(nb, t0 + nsub * L + 9, nchan, nb * 7 + L)
    _, _, sums, cnt = _long_sums(dev, x, L, nsub, t0, nchan)
    S, S2 = ccm.sums_fp64(x, L, nsub, t0)       # exact route (pinned), BLAS-fast
    assert np.array_equal(sums.cpu().numpy(), _packed(S, S2))
    assert (cnt.cpu().numpy() == L).all()
    if nb >= 3:
        assert S2[0, 0, 0, 0] > 2 ** 31         # past the int32 range


@pytest.mark.parametrize("nb,nchan,L,nsub", [(19, 24, 40960, 2), (7, 9, 203450, 1),
                                              (72, 4, 81920, 1)])
def test_long_eigen(dev, nb, nchan, L, nsub):
    import torch
    from paper_2512_16278_amd import rfi
    x = _data(nb, nsub * L, nchan, 1000 + nb)
    _, _, sums, cnt = _long_sums(dev, x, L, nsub, 0, nchan)
    ncell = nsub * nchan
    stat = torch.full((ncell,), -1.0, dtype=torch.float64, device=dev)
    status = torch.full((ncell,), 0xEE, dtype=torch.uint8, device=dev)
    ev = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
    v1 = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
    say("long eigen", nb, nchan, L, nsub)
    rfi.rfi_eig_batched_long(nb, nsub, nchan, sums, cnt, stat, status, eigvals=ev, v1=v1)
    torch.cuda.synchronize()
    cr = pipeline.cells(x, L, nsub)
    s = stat.cpu().numpy()
    st = status.cpu().numpy()
    deg = cr.degenerate.ravel()
    assert ((st & rfi.RFI_CELL_DEGENERATE) != 0).tolist() == deg.tolist()
    assert np.abs(s - cr.stat.ravel()).max() <= 1e-12
    w = cr.w.reshape(ncell, nb)
    lam1 = np.abs(w[:, 0])
    assert (np.abs(ev.cpu().numpy().T - w).max(axis=1) / lam1).max() <= 1e-6
    r = cr.r.reshape(ncell, nb, nb)
    g = v1.cpu().numpy().astype(np.float64)
    res = np.linalg.norm(np.einsum("cab,bc->ac", r, g) - w[:, 0][None, :] * g, axis=0)
    assert res.max() < 1e-5 * lam1.max()


def test_long_process_block(dev):
    import torch
    from paper_2512_16278_amd import rfi
    nb, nchan, L, nsub = 19, 40, 203450, 2
    x = _data(nb, nsub * L + 100, nchan, 7)
    buf, blk, sums, cnt = _long_sums(dev, x, L, nsub, 50, nchan)
    ncell = nsub * nchan
    stat = torch.empty(ncell, dtype=torch.float64, device=dev)
    status = torch.empty(ncell, dtype=torch.uint8, device=dev)
    rfi.rfi_eig_batched_long(nb, nsub, nchan, sums, cnt, stat, status)
    mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
    rfi.rfi_flag(nsub, nchan, stat, status, mask)
    p = rfi.process_params(L, nsub, t0=50)
    ws = torch.empty(rfi.rfi_process_workspace_size(nb, nchan, p), dtype=torch.uint8, device=dev)
    stat2 = torch.empty_like(stat)
    status2 = torch.empty_like(status)
    mask2 = torch.empty_like(mask)
    out = torch.zeros(48, dtype=torch.uint8, device=dev)
    say("long process block")
    rfi.rfi_process_block(blk, p, stat2, status2, mask2, ws, out=out)
    torch.cuda.synchronize()
    assert torch.equal(stat, stat2) and torch.equal(status, status2)
    assert torch.equal(mask, mask2)
    s = stat2.cpu().numpy()
    ref = clip.clip_iterative(s, (status2.cpu().numpy() & 17) == 0, 3.0, 50)
    fs = rfi.flag_stats_from_bytes(out.cpu().numpy().tobytes())
    assert np.array_equal(mask2.cpu().numpy().astype(bool), ref.mask)
    assert (fs["mu"], fs["sigma"], fs["thr"], fs["iterations"]) == \
        (ref.mu, ref.sigma, ref.thr, ref.iterations)
    cr = pipeline.cells(x, L, nsub, t0=50)
    assert np.abs(s - cr.stat.ravel()).max() <= 1e-12


def test_long_items_in_batch(dev):
    """A batch with a long-sub-interval item (L = 40,960, past the int32 bound)
    beside an ordinary one: every item equals rfi_process_block on its block
    alone bit for bit (statistic, status, mask, v1 and the per-beam mask of
    the long item), the long item's statistic is within 1e-12 of the oracle,
    and graph replays reproduce the eager batch."""
    import torch
    from paper_2512_16278_amd import rfi
    nb_l, nchan_l, L_l, nsub_l, t0_l = 19, 40, 40960, 2, 50
    x_l = _data(nb_l, nsub_l * L_l + 100, nchan_l, 11)
    buf_l = upload(x_l, dev)
    blk_l = rfi.make_block(buf_l, nchan_l)
    nb_s, nchan_s, L_s, nsub_s = 7, 64, 512, 8
    x_s = _data(nb_s, nsub_s * L_s, nchan_s, 12)
    buf_s = upload(x_s, dev)
    blk_s = rfi.make_block(buf_s, nchan_s)

    def outputs(nb, ncell, long_item):
        o = dict(stat=torch.full((ncell,), -1.0, dtype=torch.float64, device=dev),
                 status=torch.full((ncell,), 0xEE, dtype=torch.uint8, device=dev),
                 mask=torch.full((ncell,), 9, dtype=torch.uint8, device=dev))
        if long_item:
            o["v1"] = torch.full((nb, ncell), -9.0, dtype=torch.float32, device=dev)
            o["beam_mask"] = torch.full((nb, ncell), 9, dtype=torch.uint8, device=dev)
        return o

    items = [dict(blk=blk_l, t0=t0_l, L=L_l, nsub=nsub_l, **outputs(nb_l, nsub_l * nchan_l, True)),
             dict(blk=blk_s, t0=0, L=L_s, nsub=nsub_s, **outputs(nb_s, nsub_s * nchan_s, False))]
    bt = rfi.Batch(items)
    ws = torch.empty(bt.workspace_size(), dtype=torch.uint8, device=dev)
    say("batch with a long item")
    bt.run(ws)
    torch.cuda.synchronize()
    eager = [{k: v.clone() for k, v in it.items() if torch.is_tensor(v)} for it in items]

    # each block alone through the whole-block call
    for it, (x, nb, nchan) in zip(items, ((x_l, nb_l, nchan_l), (x_s, nb_s, nchan_s))):
        ncell = it["nsub"] * nchan
        ref = outputs(nb, ncell, "v1" in it)
        p = rfi.process_params(it["L"], it["nsub"], t0=it["t0"],
                               beam_mask=ref.get("beam_mask"))
        pws = torch.empty(rfi.rfi_process_workspace_size(nb, nchan, p), dtype=torch.uint8,
                          device=dev)
        say("whole-block call", nb, nchan, it["L"])
        rfi.rfi_process_block(it["blk"], p, ref["stat"], ref["status"], ref["mask"], pws,
                              v1=ref.get("v1"))
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], it[k]), (it["L"], k)

    cr = pipeline.cells(x_l, L_l, nsub_l, t0=t0_l)
    assert np.abs(items[0]["stat"].cpu().numpy() - cr.stat.ravel()).max() <= 1e-12

    g = bt.graph(ws)
    for rep in range(3):
        for it in items:
            for k, v in it.items():
                if torch.is_tensor(v):
                    v.fill_(7)
        say("graph replay", rep)
        g.launch()
        torch.cuda.synchronize()
        for it, ref in zip(items, eager):
            for k in ref:
                assert torch.equal(ref[k], it[k]), (rep, k)
    g.close()
