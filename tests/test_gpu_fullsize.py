"""Parity at the full FAST-shaped size (19 beams x 4096 channels, L = 2048,
99 sub-intervals, 15.78 GB), in the launch configuration the benchmark times.

The oracle cannot process all 405,504 cells in a test, so:

* sampled cells (two whole sub-intervals over 512 channels each, and eight
  channels over all 99 sub-intervals, including channels with injected
  sinusoids and the burst sub-interval) are recomputed by the FP64 oracle
  from bytes regenerated on the CPU: sums bit-exact, statistic <= 1e-9,
  status bits equal, and the mask equal to the oracle statistic against the
  GPU's final threshold;
* over every cell, properties that hold at any size: the statistic lies in
  [1/n, 1]; the mask is exactly {eligible cells with q > thr} for the
  reported fit; the reported fit is the exact moment fit of the unmasked
  eligible cells (recomputed here with Python integers, bit-equal); the clip
  reached its fixed point; and the oracle's clip over all 405,504 GPU
  statistics gives the same mask, fits and iteration count.
"""
import math

import numpy as np
import pytest

from oracle import ccm, clip, pipeline
from gpu_util import packed_oracle_sums, say

pytestmark = pytest.mark.gpu

TWO40 = float(1 << 40)


@pytest.fixture(scope="module")
def fast(request):
    import torch
    from paper_2512_16278_amd import rfi, synth
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    spec = synth.fast_spec(seconds=10.0)
    nb, nc, ns, L = spec.nbeam, spec.nchan, spec.nsamp, spec.L
    stride = (nc + 15) // 16 * 16
    say(f"full size: generating {nb} x {ns} x {nc} on the GPU")
    data = torch.empty((nb, ns, stride), dtype=torch.uint8, device=dev)
    ds = rfi.DeviceSynth(spec, dev)
    for b in range(nb):
        ds.fill(data[b], b)
    torch.cuda.synchronize()
    yield spec, data, dev
    del data
    torch.cuda.empty_cache()


def _sample_windows(spec):
    nsub = spec.nsamp // spec.L
    burst_k = [bu.t_lo // spec.L for bu in spec.bursts]
    sin_ch = sorted(s.chan for s in spec.sinusoids)
    subs = sorted({0, burst_k[0] if burst_k else nsub - 1})
    chans = sorted(set(sin_ch[:4]) | {1, 777, 2048, 4095})
    return subs, chans


def test_fullsize_process_block(fast):
    import torch
    from paper_2512_16278_amd import rfi, synth
    spec, data, dev = fast
    nb, nc, L = spec.nbeam, spec.nchan, spec.L
    nsub = spec.nsamp // L
    ncell = nsub * nc
    blk = rfi.make_block(data, nc)
    p = rfi.process_params(L, nsub)                    # the benchmark's configuration
    ws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, p), dtype=torch.uint8, device=dev)
    stat = torch.empty(ncell, dtype=torch.float64, device=dev)
    status = torch.empty(ncell, dtype=torch.uint8, device=dev)
    mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
    out = torch.zeros(48, dtype=torch.uint8, device=dev)
    say("full size: rfi_process_block")
    rfi.rfi_process_block(blk, p, stat, status, mask, ws, out=out)
    torch.cuda.synchronize()
    s = stat.cpu().numpy().reshape(nsub, nc)
    st = status.cpu().numpy().reshape(nsub, nc)
    m = mask.cpu().numpy().reshape(nsub, nc).astype(bool)
    fs = rfi.flag_stats_from_bytes(out.cpu().numpy().tobytes())
    say(f"full size: fit mu={fs['mu']:.6f} sigma={fs['sigma']:.6f} thr={fs['thr']:.6f} "
        f"iters={fs['iterations']} nflag={fs['nflag']}")

    # --- properties over every cell -------------------------------------------------
    elig = (st & (rfi.RFI_CELL_DEGENERATE | rfi.RFI_CELL_BAD_COUNT)) == 0
    assert elig.all()                                   # no degenerate cells in this data
    assert (s >= 1.0 / nb - 1e-12).all() and (s <= 1.0 + 1e-12).all()
    q = np.rint(s * TWO40).astype(np.int64)
    assert fs["converged"] == 1 and 1 <= fs["iterations"] <= 50
    T = math.floor(fs["thr"] * TWO40)
    assert np.array_equal(m, elig & (q > T))
    assert fs["nflag"] == int(m.sum())
    live = [int(v) for v in q[elig & ~m]]
    N, Q1, Q2 = len(live), sum(live), sum(v * v for v in live)
    assert fs["nfit"] == N
    mu = Q1 / (N << 40)
    var = (N * Q2 - Q1 * Q1) / ((N * N) << 80)
    assert fs["mu"] == mu and fs["sigma"] == math.sqrt(var)       # one rounding each
    assert fs["thr"] == mu + 3.0 * math.sqrt(var)
    # the oracle's clip over every cell's GPU statistic: the same mask and fits
    say("full size: oracle clip over all cells")
    ref = clip.clip_iterative(s.ravel(), elig.ravel(), 3.0, 50)
    assert np.array_equal(m.ravel(), ref.mask)
    assert (fs["mu"], fs["sigma"], fs["thr"], fs["iterations"], fs["nflag"]) == \
        (ref.mu, ref.sigma, ref.thr, ref.iterations, ref.nflag)
    # fixed point: the last fit masks nothing new
    assert (q[elig & ~m] * 2.0 ** -40 <= fs["thr"]).all()
    # every injected common-mode channel is masked in most sub-intervals
    for sn in spec.sinusoids:
        assert m[:, sn.chan].mean() > 0.9, sn.chan

    # --- sampled cells against the oracle -------------------------------------------
    subs, chans = _sample_windows(spec)
    thr = fs["thr"]
    for k in subs:
        say(f"full size: oracle on sub-interval {k}, channels 0..511")
        x = synth.generate(spec, k * L, (k + 1) * L, 0, 512)
        cr, _, _ = pipeline.block(x, L, 1)
        so = cr.stat.ravel()
        assert np.abs(s[k, :512] - so).max() <= 1e-9, k
        qo = np.rint(so * TWO40) * 2.0 ** -40
        clear = np.abs(qo - thr) > 1e-9
        assert np.array_equal(m[k, :512][clear], (qo > thr)[clear]), k
    for c in chans:
        say(f"full size: oracle on channel {c}, all sub-intervals")
        x = synth.generate(spec, 0, nsub * L, c, c + 1)
        cr, _, _ = pipeline.block(x, L, nsub)
        so = cr.stat.ravel()
        assert np.abs(s[:, c] - so).max() <= 1e-9, c
        qo = np.rint(so * TWO40) * 2.0 ** -40
        clear = np.abs(qo - thr) > 1e-9
        assert np.array_equal(m[:, c][clear], (qo > thr)[clear]), c


def test_fullsize_sums_sampled(fast):
    import torch
    from paper_2512_16278_amd import rfi, synth
    spec, data, dev = fast
    nb, nc, L = spec.nbeam, spec.nchan, spec.L
    nsub = spec.nsamp // L
    ncell = nsub * nc
    npair = nb * (nb + 1) // 2
    blk = rfi.make_block(data, nc)
    sx = torch.empty((nb, ncell), dtype=torch.int32, device=dev)
    sxy = torch.empty((npair, ncell), dtype=torch.int32, device=dev)
    cnt = torch.empty(nsub, dtype=torch.int32, device=dev)
    say("full size: rfi_ccm_accumulate (MFMA)")
    rfi.rfi_ccm_accumulate(blk, 0, L, nsub, sx, sxy, cnt, variant=rfi.RFI_CCM_MFMA)
    torch.cuda.synchronize()
    assert (cnt.cpu().numpy() == L).all()
    gx = sx.cpu().numpy().reshape(nb, nsub, nc)
    gxy = sxy.cpu().numpy().reshape(npair, nsub, nc)
    subs, chans = _sample_windows(spec)
    for k in subs:
        x = synth.generate(spec, k * L, (k + 1) * L, 0, 512)
        S, S2 = ccm.sums_fp64(x, L, 1)
        rx, rxy = packed_oracle_sums(S, S2)
        assert np.array_equal(gx[:, k, :512], rx), k
        assert np.array_equal(gxy[:, k, :512], rxy), k
    for c in chans[:3]:
        x = synth.generate(spec, 0, nsub * L, c, c + 1)
        S, S2 = ccm.sums_fp64(x, L, nsub)
        rx, rxy = packed_oracle_sums(S, S2)
        assert np.array_equal(gx[:, :, c], rx), c
        assert np.array_equal(gxy[:, :, c], rxy), c


def test_fullsize_eigvec_stage(fast):
    """The per-beam eigenvector stage (Sec. 3.3 last paragraph; kappa_v = 1)
    on the whole FAST-shaped block, in the benchmark's launch configuration:
    v1 of the whole-block call against the oracle on the sampled cells (up to
    sign where sum(v1) ~ 0, where the gap lambda_1 - lambda_2 is clear), and
    over every cell the per-beam fits and masks against the same moment fit
    recomputed here in FP64 from the GPU's v1 and mask."""
    import torch
    from paper_2512_16278_amd import rfi, synth
    spec, data, dev = fast
    nb, nc, L = spec.nbeam, spec.nchan, spec.L
    nsub = spec.nsamp // L
    ncell = nsub * nc
    blk = rfi.make_block(data, nc)
    p = rfi.process_params(L, nsub)
    ws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, p), dtype=torch.uint8, device=dev)
    stat = torch.empty(ncell, dtype=torch.float64, device=dev)
    status = torch.empty(ncell, dtype=torch.uint8, device=dev)
    mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
    v1 = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
    bmask = torch.empty((nb, ncell), dtype=torch.uint8, device=dev)
    bmu = torch.empty(nb, dtype=torch.float64, device=dev)
    bsd = torch.empty(nb, dtype=torch.float64, device=dev)
    say("full size: rfi_process_block with v1, then rfi_eigvec_flag")
    rfi.rfi_process_block(blk, p, stat, status, mask, ws, v1=v1)
    rfi.rfi_eigvec_flag(nb, nsub, nc, v1, mask, status, bmask, kappa_v=1.0, beam_mu=bmu,
                        beam_sigma=bsd)
    torch.cuda.synchronize()
    g = v1.cpu().numpy().reshape(nb, nsub, nc)
    m = mask.cpu().numpy().astype(bool)
    bm = bmask.cpu().numpy().astype(bool)
    assert np.allclose(np.linalg.norm(g, axis=0), 1.0, atol=1e-5)
    # sampled cells against the oracle's v1
    subs, chans = _sample_windows(spec)
    for k in subs:
        say(f"full size: oracle v1 on sub-interval {k}")
        x = synth.generate(spec, k * L, (k + 1) * L, 0, 512)
        cr = pipeline.cells(x, L, 1)
        vo = cr.v1.reshape(512, nb)
        w = cr.w.reshape(512, nb)
        vg = g[:, k, :512].T.astype(np.float64)
        clear = (w[:, 0] - w[:, 1]) / np.abs(w[:, 0]) > 0.05
        tie = np.abs(vo.sum(axis=1)) < 1e-5
        d = np.where(tie[:, None], np.minimum(np.abs(vg - vo), np.abs(vg + vo)), np.abs(vg - vo))
        assert d.max(axis=1)[clear].max() < 1e-4, k
    # every cell: the per-beam moment fit of |v1_b| over eligible unmasked cells
    a = np.abs(g.reshape(nb, ncell).astype(np.float64))
    clean = ~m
    mu = a[:, clean].mean(axis=1)
    sd = np.sqrt(((a[:, clean] - mu[:, None]) ** 2).mean(axis=1))
    gmu, gsd = bmu.cpu().numpy(), bsd.cpu().numpy()
    assert np.abs(gmu - mu).max() <= 1e-12 * mu.max()
    assert np.abs(gsd - sd).max() <= 1e-10 * sd.max()
    thr = (gmu + gsd)[:, None]
    ref = m[None, :] & (a > thr)
    assert np.array_equal(bm, ref)
    assert not (bm & ~m[None, :]).any()
    assert bm.any(axis=0)[m].mean() > 0.3       # most flagged cells name their beams


def test_fullsize_one_10s_sub_interval(fast):
    """Table 1's longest sub-interval: the whole 10 s FAST-shaped block as one
    sub-interval of L = 203,450 samples (int64 sums in time chunks), 4096
    cells: sampled channels against the oracle (statistic within 1e-12) and
    the clip against the oracle's clip of the same statistic (bit-equal)."""
    import torch
    from paper_2512_16278_amd import rfi, synth
    spec, data, dev = fast
    nb, nc = spec.nbeam, spec.nchan
    L = spec.nsamp
    blk = rfi.make_block(data, nc)
    p = rfi.process_params(L, 1)
    ws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, p), dtype=torch.uint8, device=dev)
    stat = torch.empty(nc, dtype=torch.float64, device=dev)
    status = torch.empty(nc, dtype=torch.uint8, device=dev)
    mask = torch.empty(nc, dtype=torch.uint8, device=dev)
    out = torch.zeros(48, dtype=torch.uint8, device=dev)
    say(f"full size: one sub-interval of {L} samples")
    rfi.rfi_process_block(blk, p, stat, status, mask, ws, out=out)
    torch.cuda.synchronize()
    s = stat.cpu().numpy()
    m = mask.cpu().numpy().astype(bool)
    fs = rfi.flag_stats_from_bytes(out.cpu().numpy().tobytes())
    ref = clip.clip_iterative(s, (status.cpu().numpy() & 17) == 0, 3.0, 50)
    assert np.array_equal(m, ref.mask)
    assert (fs["mu"], fs["sigma"], fs["thr"], fs["iterations"]) == \
        (ref.mu, ref.sigma, ref.thr, ref.iterations)
    _, chans = _sample_windows(spec)
    for c in chans:
        say(f"full size: oracle on channel {c}, L = {L}")
        x = synth.generate(spec, 0, L, c, c + 1)
        cr = pipeline.cells(x, L, 1)
        assert abs(s[c] - cr.stat[0, 0]) <= 1e-12, c
    for sn in spec.sinusoids[:8]:
        assert m[sn.chan], sn.chan                      # persistent common-mode channels
