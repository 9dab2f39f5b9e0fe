"""GPU: the whole-block call rfi_process_block (sums -> eigen -> clip, with
sub-interval groups pipelined over two streams).

Its outputs must equal those of the three separate calls bit for bit (same
arithmetic, different tiling and launch shapes only), and the statistic and
mask must meet the oracle at the tolerances of the separate calls: stat within
1e-9 (FP32 Jacobi + FP64 Rayleigh quotient), masks identical.
"""
import numpy as np
import pytest

from gpu_util import eig_buffers, say, sums_buffers, upload
from oracle import clip, pipeline

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_16278_amd import rfi
    rfi.lib()
    return torch.device("cuda:0")


def _data(nbeam, nchan, nsamp, seed):
    """Noise with a common-mode sinusoid in a few channels (correlated beams)."""
    rng = np.random.default_rng(seed)
    x = 128 + 20 * rng.standard_normal((nbeam, nsamp, nchan))
    t = np.arange(nsamp)
    for j in rng.choice(nchan, size=max(1, nchan // 40), replace=False):
        g = rng.uniform(0.5, 1.5, nbeam)
        x[:, :, j] += 12 * g[:, None] * np.sin(2 * np.pi * t / 37.0 + j)[None, :]
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def _state(dev):
    import torch
    from paper_2512_16278_amd import rfi
    return torch.zeros(len(bytes(rfi.rfi_stream_state())), dtype=torch.uint8, device=dev)


def _separate(blk, nb, nc, t0, L, nsub, dev, precision, state=None, vectors=False):
    import torch
    from paper_2512_16278_amd import rfi
    sx, sxy, cnt = sums_buffers(nb, nsub, nc, dev)
    stat, status, ev, v1 = eig_buffers(nb, nsub * nc, dev, with_vectors=vectors)
    mask = torch.full((nsub * nc,), 7, dtype=torch.uint8, device=dev)
    out = torch.zeros(48, dtype=torch.uint8, device=dev)
    rfi.rfi_ccm_accumulate(blk, t0, L, nsub, sx, sxy, cnt)
    rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, eigvals=ev, v1=v1,
                        precision=precision)
    rfi.rfi_flag(nsub, nc, stat, status, mask, state=state, out=out)
    torch.cuda.synchronize()
    return stat, status, mask, out, ev, v1


def _process(blk, nb, nc, t0, L, nsub, dev, precision, group, state=None, vectors=False):
    import torch
    from paper_2512_16278_amd import rfi
    p = rfi.process_params(L, nsub, t0=t0, group=group, eig_precision=precision)
    nws = rfi.rfi_process_workspace_size(nb, nc, p)
    assert nws > 0
    ws = torch.empty(nws, dtype=torch.uint8, device=dev)
    stat, status, ev, v1 = eig_buffers(nb, nsub * nc, dev, with_vectors=vectors)
    mask = torch.full((nsub * nc,), 7, dtype=torch.uint8, device=dev)
    out = torch.zeros(48, dtype=torch.uint8, device=dev)
    rfi.rfi_process_block(blk, p, stat, status, mask, ws, state=state, eigvals=ev, v1=v1,
                          out=out)
    torch.cuda.synchronize()
    return stat, status, mask, out, ev, v1


CASES = [
    # nbeam, nchan, L, nsub, t0, precision, group
    (19, 200, 256, 7, 3, 32, 0),
    (19, 200, 256, 7, 0, 32, 1),
    (19, 200, 256, 7, 0, 32, 3),
    (19, 4096, 64, 9, 0, 32, 2),
    (7, 97, 128, 5, 1, 32, 2),
    (36, 65, 300, 4, 0, 32, 3),
    (19, 64, 512, 3, 0, 64, 1),
]


@pytest.mark.parametrize("nb,nc,L,nsub,t0,prec,group", CASES)
def test_process_block_equals_separate_calls(dev, nb, nc, L, nsub, t0, prec, group):
    from paper_2512_16278_amd import rfi
    x = _data(nb, nc, t0 + nsub * L + 11, seed=nb * 7 + nc + L)
    buf = upload(x, dev)
    blk = rfi.make_block(buf, nc)
    vec = nb * nc * nsub <= 200000
    say("process_block", nb, nc, L, nsub, t0, prec, group)
    a = _separate(blk, nb, nc, t0, L, nsub, dev, prec, vectors=vec)
    b = _process(blk, nb, nc, t0, L, nsub, dev, prec, group, vectors=vec)
    for i, name in enumerate(("stat", "status", "mask", "out", "eigvals", "v1")):
        if a[i] is None:
            continue
        assert np.array_equal(a[i].cpu().numpy(), b[i].cpu().numpy()), name


def test_process_block_vs_oracle(dev):
    from paper_2512_16278_amd import rfi
    nb, nc, L, nsub = 19, 96, 512, 6
    x = _data(nb, nc, nsub * L, seed=11)
    buf = upload(x, dev)
    blk = rfi.make_block(buf, nc)
    say("process_block vs oracle")
    stat, status, mask, out, _, _ = _process(blk, nb, nc, 0, L, nsub, dev, 32, 2)
    cr, res, _ = pipeline.block(x, L, nsub)
    s = stat.cpu().numpy()
    assert np.abs(s - cr.stat.ravel()).max() <= 1e-9
    assert np.array_equal(mask.cpu().numpy().astype(bool), res.mask.ravel())
    st = rfi.flag_stats_from_bytes(out.cpu().numpy().tobytes())
    assert st["iterations"] == res.iterations and st["nflag"] == res.nflag


def test_process_block_stream_state(dev):
    """Three blocks of one stream through the pooled clip state, against the
    separate calls and the oracle's pooled clip."""
    from paper_2512_16278_amd import rfi
    nb, nc, L = 19, 128, 256
    sa, sb = _state(dev), _state(dev)
    ost = clip.StreamState()
    for i in range(3):
        nsub = 3 + i
        x = _data(nb, nc, nsub * L, seed=100 + i)
        buf = upload(x, dev)
        blk = rfi.make_block(buf, nc)
        say("process_block stream block", i)
        a = _separate(blk, nb, nc, 0, L, nsub, dev, 32, state=sa)
        b = _process(blk, nb, nc, 0, L, nsub, dev, 32, 2, state=sb)
        for j in range(4):
            assert np.array_equal(a[j].cpu().numpy(), b[j].cpu().numpy()), (i, j)
        cr = pipeline.cells(x, L, nsub)
        ref = clip.clip_stream(ost, cr.stat.ravel(), ~cr.degenerate.ravel())
        assert np.array_equal(b[2].cpu().numpy().astype(bool), ref.mask)
        assert np.abs(b[0].cpu().numpy() - cr.stat.ravel()).max() <= 1e-9
    assert np.array_equal(sa.cpu().numpy(), sb.cpu().numpy())


def test_process_block_beam_mask(dev):
    """The per-beam stage inside the whole-block call (Sec. 3.3 last
    paragraph): bit-equal to rfi_eigvec_flag on the call's own v1 and mask,
    and against the oracle's stage on the same cells (identical except where
    |v1_b| lies within FP32 resolution of the beam's threshold). Both
    precisions, a 36-beam block on the tridiagonal solver, and the error when
    v1 is not requested."""
    import torch
    from paper_2512_16278_amd import rfi
    from oracle import eigvec
    for nb, nc, L, nsub, prec in ((19, 96, 512, 6, 32), (19, 64, 256, 4, 64), (36, 40, 300, 3, 32)):
        x = _data(nb, nc, nsub * L, seed=nb + nc)
        buf = upload(x, dev)
        blk = rfi.make_block(buf, nc)
        ncell = nsub * nc
        bm = torch.full((nb, ncell), 7, dtype=torch.uint8, device=dev)
        p = rfi.process_params(L, nsub, eig_precision=prec, kappa_v=1.0, beam_mask=bm)
        ws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, p), dtype=torch.uint8, device=dev)
        stat, status, _, v1 = eig_buffers(nb, ncell, dev)
        mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
        say("process_block beam mask", nb, nc, L, nsub, prec)
        rfi.rfi_process_block(blk, p, stat, status, mask, ws, v1=v1)
        bm2 = torch.full((nb, ncell), 9, dtype=torch.uint8, device=dev)
        rfi.rfi_eigvec_flag(nb, nsub, nc, v1, mask, status, bm2, kappa_v=1.0)
        torch.cuda.synchronize()
        g = bm.cpu().numpy()
        assert set(np.unique(g)) <= {0, 1}
        assert np.array_equal(g, bm2.cpu().numpy())
        cr, res, bo = pipeline.block(x, L, nsub, kappa_v=1.0)
        assert np.array_equal(mask.cpu().numpy().astype(bool), res.mask.ravel())
        diff = g.astype(bool) != bo.reshape(nb, -1)
        if diff.any():
            ok = ~cr.degenerate.ravel()
            _, mu, sd = eigvec.eigvec_mask(cr.v1.reshape(-1, nb), res.mask.ravel(), ok, 1.0)
            a = np.abs(cr.v1.reshape(-1, nb)).T
            assert (np.abs(a - (mu + sd)[:, None])[diff] < 1e-5).all()
        assert g[:, ~res.mask.ravel()].sum() == 0          # only masked cells carry beam flags
    p = rfi.process_params(L, nsub, beam_mask=bm)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_process_block(blk, p, stat, status, mask, ws)            # no v1 output
    p = rfi.process_params(L, nsub, kappa_v=-1.0, beam_mask=bm)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_process_block(blk, p, stat, status, mask, ws, v1=v1)


@pytest.mark.parametrize("scopes,fit", [(7, 0), (7, 1), (2, 1), (0, 1), (4, 0)])
def test_process_block_scoped_clip(dev, scopes, fit):
    """The whole-block call with the clip scopes / histogram fit of Sec. 3.3
    (rfi_flag_scoped's clip on the call's own statistic): mask and global
    summary bit-equal to rfi_flag_scoped run after the call; stat and status
    unchanged by the choice; a pooled state is refused with scopes."""
    import torch
    from paper_2512_16278_amd import rfi
    nb, nc, L, nsub = 19, 96, 256, 9
    x = _data(nb, nc, nsub * L, seed=17)
    buf = upload(x, dev)
    blk = rfi.make_block(buf, nc)
    p = rfi.process_params(L, nsub, scopes=scopes, fit=fit)
    ws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, p), dtype=torch.uint8, device=dev)
    stat, status, _, _ = eig_buffers(nb, nsub * nc, dev, with_vectors=False)
    mask = torch.full((nsub * nc,), 7, dtype=torch.uint8, device=dev)
    out = torch.zeros(48, dtype=torch.uint8, device=dev)
    say("process_block scoped", scopes, fit)
    rfi.rfi_process_block(blk, p, stat, status, mask, ws, out=out)
    m2 = torch.full_like(mask, 9)
    out2 = torch.zeros_like(out)
    rfi.rfi_flag_scoped(nsub, nc, stat, status, m2, scopes=scopes or rfi.RFI_SCOPE_GLOBAL, fit=fit,
                        out=out2)
    torch.cuda.synchronize()
    assert np.array_equal(mask.cpu().numpy(), m2.cpu().numpy())
    if (scopes or 1) & 1:
        assert np.array_equal(out.cpu().numpy(), out2.cpu().numpy())
    a = _separate(blk, nb, nc, 0, L, nsub, dev, 32)
    assert np.array_equal(a[0].cpu().numpy(), stat.cpu().numpy())
    assert np.array_equal(a[1].cpu().numpy(), status.cpu().numpy())
    st = _state(dev)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_process_block(blk, p, stat, status, mask, ws, state=st)


def test_process_block_empty_and_errors(dev):
    import torch
    from paper_2512_16278_amd import rfi
    nb, nc, L = 19, 64, 128
    x = _data(nb, nc, 2 * L, seed=3)
    buf = upload(x, dev)
    blk = rfi.make_block(buf, nc)
    say("process_block empty / errors")
    st = _process(blk, nb, nc, 0, L, 0, dev, 32, 0)
    assert (st[1].cpu().numpy() == 0xEE).all()          # nothing written for nsub = 0
    p = rfi.process_params(L, 3)                          # 3 sub-ints do not fit
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev)
    stat, status, _, _ = eig_buffers(nb, 3 * nc, dev, with_vectors=False)
    mask = torch.empty(3 * nc, dtype=torch.uint8, device=dev)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_process_block(blk, p, stat, status, mask, ws)
    p = rfi.process_params(L, 2)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_process_block(blk, p, stat, status, mask, None)
