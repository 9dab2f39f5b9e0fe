"""GPU: ArPLS bandpass (Sec. 3.1, parameters of Sec. 4.5) and the non-centred
CCM of the bandpass-subtracted power, against the oracle.

* rfi_bandpass_arpls: the GPU's banded Cholesky and the oracle's dense solve
  round differently; A = W + lam D^T D has a condition number of order
  16 lam / min(eig W restricted to linear functions) ~ 1e6 - 1e7 here, so the
  baselines agree to 1e-8 of the spectrum's scale and the pass counts are
  identical (no ratio test lies within that distance of its threshold in these
  data). Edge cases: fewer than 3 channels (z = y, no pass), exactly 3, a
  flat spectrum, itermax = 1, no passes output.
* rfi_eig_noncentred: given the same z, every matrix entry is formed in the
  oracle's order, so the statistic agrees to 1e-12 (the solvers differ) and
  the eigenvalues to 1e-6 of lambda_1; the whole chain (GPU sums -> GPU z ->
  statistic) against the oracle's own chain to 1e-6, the z rounding carried
  through the cancellation S_ab - z S_a - ...; degenerate (M = 0) and bad
  count cells flagged.
"""
import numpy as np
import pytest

from gpu_util import say, sums_buffers, upload
from oracle import bandpass, ccm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_16278_amd import rfi
    rfi.lib()
    return torch.device("cuda:0")


def _spectra(rng, nbeam, nsub, F):
    """Channel means of FAST-like bandpasses: a smooth passband per beam, noise
    and positive RFI spikes in a few channels."""
    j = np.arange(F)
    y = np.empty((nsub, F, nbeam))
    for b in range(nbeam):
        base = 90 + 40 * np.sin(np.pi * (j + 0.5) / F) ** 0.6 + 6 * np.cos(2 * np.pi * j / (F / 3 + 1))
        base *= rng.uniform(0.8, 1.2)
        for k in range(nsub):
            v = base + 0.8 * rng.standard_normal(F)
            hot = rng.choice(F, size=max(1, F // 40), replace=False)
            v[hot] += rng.uniform(5, 60, size=hot.size)
            y[k, :, b] = v
    return y


def _run_arpls(dev, S, L, lam=1e5, ratio=0.05, itermax=100, with_passes=True):
    import torch
    from paper_2512_16278_amd import rfi
    nsub, F, nb = S.shape
    sx = torch.from_numpy(np.ascontiguousarray(S.reshape(nsub * F, nb).T.astype(np.int32))).to(dev)
    cnt = torch.from_numpy(np.asarray(L, dtype=np.int32)).to(dev)
    z = torch.full((nb, nsub * F), -7.0, dtype=torch.float64, device=dev)
    passes = torch.full((nsub, nb), -7, dtype=torch.int32, device=dev) if with_passes else None
    say("arpls", nb, nsub, F, lam, ratio, itermax)
    rfi.rfi_bandpass_arpls(nb, nsub, F, sx, cnt, z, passes=passes, lam=lam, ratio=ratio,
                           itermax=itermax)
    torch.cuda.synchronize()
    zg = z.cpu().numpy().reshape(nb, nsub, F).transpose(1, 2, 0)
    return zg, (passes.cpu().numpy() if with_passes else None)


@pytest.mark.parametrize("nb,nsub,F,lam,ratio,itermax", [
    (3, 2, 64, 1e5, 0.05, 100), (19, 3, 257, 1e5, 0.05, 100), (3, 1, 1000, 1e6, 0.01, 100),
    (2, 4, 3, 1e5, 0.05, 100), (4, 2, 37, 1e3, 0.05, 1), (7, 2, 130, 1e4, 0.001, 30)])
def test_arpls_matches_oracle(dev, nb, nsub, F, lam, ratio, itermax):
    rng = np.random.default_rng(nb * 1000 + F)
    y = _spectra(rng, nb, nsub, F)
    L = rng.integers(800, 1100, size=nsub)
    S = np.rint(y * L[:, None, None]).astype(np.int64)
    zg, pg = _run_arpls(dev, S, L, lam, ratio, itermax)
    zo, po = bandpass.bandpass_from_sums(S, L, lam, ratio, itermax)
    scale = np.abs(S / L[:, None, None]).max()
    assert np.abs(zg - zo).max() <= 1e-8 * scale
    assert np.array_equal(pg, po)
    assert (po >= 1).all() and (po <= itermax).all()


def test_arpls_edge_cases(dev):
    rng = np.random.default_rng(5)
    # fewer than three channels: the baseline is the spectrum itself
    for F in (1, 2):
        S = rng.integers(1000, 200000, size=(3, F, 2))
        L = np.array([1000, 999, 1001])
        zg, pg = _run_arpls(dev, S, L)
        assert np.array_equal(zg, S / L[:, None, None])
        assert (pg == 0).all()
    # a flat spectrum: z = y solves every pass exactly, so both sides land
    # within rounding of it (the oracle's dense solve is 2.6e-9 off here)
    S = np.full((2, 50, 3), 123456, dtype=np.int64)
    zg, _ = _run_arpls(dev, S, np.array([1000, 1000]))
    assert np.abs(zg - 123.456).max() <= 1e-8 * 123.456
    # without the passes output
    y = _spectra(rng, 5, 2, 80)
    L = np.array([1024, 1024])
    S = np.rint(y * 1024).astype(np.int64)
    zg, _ = _run_arpls(dev, S, L, with_passes=False)
    zo, _ = bandpass.bandpass_from_sums(S, L)
    assert np.abs(zg - zo).max() <= 1e-8 * np.abs(y).max()


def test_arpls_rejects_bad_arguments(dev):
    import torch
    from paper_2512_16278_amd import rfi
    sx = torch.zeros((2, 8), dtype=torch.int32, device=dev)
    cnt = torch.ones(1, dtype=torch.int32, device=dev)
    z = torch.zeros((2, 8), dtype=torch.float64, device=dev)
    for kw in ({"lam": 0.0}, {"ratio": -1.0}, {"itermax": 0}):
        with pytest.raises(rfi.RfiError):
            rfi.rfi_bandpass_arpls(2, 1, 8, sx, cnt, z, **kw)
    with pytest.raises(rfi.RfiError):
        rfi.rfi_bandpass_arpls(1, 1, 8, sx, cnt, z)


def _data(rng, nb, nsamp, F):
    j = np.arange(F)
    bp = 80 + 50 * np.sin(np.pi * (j + 0.5) / F)
    x = bp[None, None, :] + 20 * rng.standard_normal((nb, nsamp, F))
    t = np.arange(nsamp)
    x[:, :, F // 3] += 30 * rng.uniform(0.2, 1.0, nb)[:, None] * np.sin(2 * np.pi * t / 50.0)[None, :]
    x[: nb // 2, nsamp // 3: nsamp // 3 + 40, :] += 60                # broadband burst
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def _gpu_sums(dev, x, L, nsub, F):
    import torch
    from paper_2512_16278_amd import rfi
    nb = x.shape[0]
    buf = upload(x, dev)
    blk = rfi.make_block(buf, F)
    sx, sxy, cnt = sums_buffers(nb, nsub, F, dev)
    say("sums", nb, nsub, F, L)
    rfi.rfi_ccm_accumulate(blk, 0, L, nsub, sx, sxy, cnt)
    torch.cuda.synchronize()
    return buf, sx, sxy, cnt


def _noncentred(dev, nb, nsub, F, sx, sxy, cnt, z):
    import torch
    from paper_2512_16278_amd import rfi
    ncell = nsub * F
    stat = torch.full((ncell,), -1.0, dtype=torch.float64, device=dev)
    status = torch.full((ncell,), 0xEE, dtype=torch.uint8, device=dev)
    ev = torch.full((nb, ncell), -9.0, dtype=torch.float32, device=dev)
    v1 = torch.full((nb, ncell), -9.0, dtype=torch.float32, device=dev)
    say("noncentred", nb, nsub, F, z is not None)
    rfi.rfi_eig_noncentred(nb, nsub, F, sx, sxy, cnt, z, stat, status, eigvals=ev, v1=v1)
    torch.cuda.synchronize()
    return stat.cpu().numpy(), status.cpu().numpy(), ev.cpu().numpy(), v1.cpu().numpy()


@pytest.mark.parametrize("nb,nsub,F,L", [(19, 3, 96, 1024), (7, 2, 41, 4096), (36, 2, 17, 512),
                                         (72, 1, 9, 2000)])
def test_noncentred_statistic(dev, nb, nsub, F, L):
    import torch
    from paper_2512_16278_amd import rfi
    rng = np.random.default_rng(nb + 31 * F)
    x = _data(rng, nb, nsub * L, F)
    _, sx, sxy, cnt = _gpu_sums(dev, x, L, nsub, F)
    S, S2 = ccm.sums_fp64(x, L, nsub)
    z = torch.empty((nb, nsub * F), dtype=torch.float64, device=dev)
    rfi.rfi_bandpass_arpls(nb, nsub, F, sx, cnt, z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy().reshape(nb, nsub, F).transpose(1, 2, 0)
    for zt, zo in ((z, zg), (None, np.zeros_like(zg))):
        s, st, ev, v1 = _noncentred(dev, nb, nsub, F, sx, sxy, cnt, zt)
        M = bandpass.noncentred_ccm(S, S2, L, zo)                     # [k, j, a, b]
        so, _ = bandpass.statistic_general(M)
        assert (st == 0).all()
        assert np.abs(s - so.ravel()).max() <= 1e-12
        w = np.linalg.eigvalsh(M).reshape(nsub * F, nb)
        order = np.argsort(-np.abs(w), axis=1, kind="stable")
        w = np.take_along_axis(w, order, axis=1)
        lam1 = np.abs(w[:, 0])
        assert (np.abs(ev.T - w).max(axis=1) / lam1).max() <= 1e-6
        Mc = M.reshape(nsub * F, nb, nb)
        g = v1.astype(np.float64)
        res = np.linalg.norm(np.einsum("cab,bc->ac", Mc, g) - w[:, 0][None, :] * g, axis=0)
        assert (res / lam1).max() < 1e-5
    # the whole chain against the oracle's own: z from the oracle's ArPLS
    zo, _ = bandpass.bandpass_from_sums(S, L)
    so, _ = bandpass.statistic_general(bandpass.noncentred_ccm(S, S2, L, zo))
    s, _, _, _ = _noncentred(dev, nb, nsub, F, sx, sxy, cnt, z)
    assert np.abs(s - so.ravel()).max() <= 1e-6
    # without the bandpass the mean dominates: a rank-one matrix, statistic near 1
    s0, _, _, _ = _noncentred(dev, nb, nsub, F, sx, sxy, cnt, None)
    assert s0.min() > 0.9 and s.mean() < s0.mean()


def test_noncentred_degenerate_and_bad_count(dev):
    nb, nsub, F, L = 5, 3, 8, 256
    rng = np.random.default_rng(9)
    x = _data(rng, nb, nsub * L, F)
    x[:, :, 2] = 0                                   # M = 0 with z = 0
    _, sx, sxy, cnt = _gpu_sums(dev, x, L, nsub, F)
    s, st, _, _ = _noncentred(dev, nb, nsub, F, sx, sxy, cnt, None)
    st = st.reshape(nsub, F)
    assert (st[:, 2] & 1).all() and (st[:, [0, 1, 3, 4, 5, 6, 7]] == 0).all()
    assert (s.reshape(nsub, F)[:, 2] == 0).all()
    cnt2 = cnt.clone()
    cnt2[1] = 1
    s, st, _, _ = _noncentred(dev, nb, nsub, F, sx, sxy, cnt2, None)
    st = st.reshape(nsub, F)
    assert (st[1] & 16).all() and ((st[[0, 2]] & 16) == 0).all()


def test_arpls_full_band(dev):
    """19 beams x 4096 channels (the FAST configuration), one sub-interval of
    1024 samples: every system on the GPU, beam 0 against the dense oracle
    (three passes: each dense 4096 x 4096 solve takes seconds on the CPU)."""
    nb, F = 19, 4096
    rng = np.random.default_rng(4096)
    y = _spectra(rng, nb, 1, F)
    L = np.array([1024])
    S = np.rint(y * 1024).astype(np.int64)
    zg, pg = _run_arpls(dev, S, L, itermax=3)
    z0, p0 = bandpass.arpls(S[0, :, 0] / 1024.0, itermax=3)
    assert np.abs(zg[0, :, 0] - z0).max() <= 1e-8 * np.abs(y).max()
    assert pg[0, 0] == p0
    assert np.isfinite(zg).all() and (pg >= 1).all()
