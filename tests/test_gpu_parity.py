"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (derived from the arithmetic of each step):
* sums: bit-exact (integer).
* eigenvalues from FP32 Jacobi: |d lambda_i| <= 1e-5 * lambda_1 (norm-relative);
  the FP64 Jacobi: 1e-6 (the output array is FP32).
* statistic lambda_1^2 / ||C||_F^2 with the FP64 Rayleigh refinement: |ds| <= 1e-9
  (an FP32 eigenvector gives a Rayleigh quotient error of order
  ||dC||^2 / gap ~ 1e-11 .. 1e-9 for the gaps of noise cells);
  FP64 Jacobi: 1e-12.
* masks: identical (both sides decide s_q > thr in FP64).
"""
import math

import numpy as np
import pytest

from gpu_util import eig_buffers, packed_oracle_sums, say, sums_buffers, upload
from oracle import ccm, clip, eig, eigvec, pipeline

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_16278_amd import rfi
    rfi.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def tiny():
    from paper_2512_16278_amd import synth
    spec = synth.tiny_spec()
    return spec, synth.generate(spec)


def run_ccm(x, L, nsub, dev, variant=0, t0=0, stride=None, nchan=None):
    import torch
    from paper_2512_16278_amd import rfi
    nb, nt, nc = x.shape
    buf = upload(x, dev, stride)
    blk = rfi.make_block(buf, nc)
    sx, sxy, cnt = sums_buffers(nb, nsub, nc, dev)
    rfi.rfi_ccm_accumulate(blk, t0, L, nsub, sx, sxy, cnt, variant=variant)
    torch.cuda.synchronize()
    return sx.cpu().numpy(), sxy.cpu().numpy(), cnt.cpu().numpy(), (buf, blk, sx, sxy, cnt)


def test_ccm_staggered_placement(dev, tiny):
    """Beams placed by rfi_beam_offsets give the oracle's sums bit for bit
    (placement is a speed matter only)."""
    import torch
    from paper_2512_16278_amd import rfi
    spec, x = tiny
    nb, nt, nc = x.shape
    L, nsub = spec.L, spec.nsamp // spec.L
    say("ccm staggered placement", nb, nt, nc)
    raw, beams = rfi.alloc_beams(nb, nt, 64, dev)
    for b in range(nb):
        assert beams[b].data_ptr() % 4096 == 64 * b
        beams[b][:, :nc].copy_(torch.from_numpy(np.ascontiguousarray(x[b])).to(dev))
    blk = rfi.make_block(beams, nc)
    sx, sxy, cnt = sums_buffers(nb, nsub, nc, dev)
    rfi.rfi_ccm_accumulate(blk, 0, L, nsub, sx, sxy, cnt)
    torch.cuda.synchronize()
    S, S2 = ccm.sums_fp64(x, L, nsub)
    rsx, rsxy = packed_oracle_sums(S, S2)
    assert np.array_equal(sx.cpu().numpy(), rsx)
    assert np.array_equal(sxy.cpu().numpy(), rsxy)


@pytest.mark.parametrize("variant", [1, 2])
def test_ccm_tiny_bit_exact(dev, tiny, variant):
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    say("ccm tiny variant", variant)
    sx, sxy, cnt, _ = run_ccm(x, L, nsub, dev, variant)
    S, S2 = ccm.sums_fp64(x, L, nsub)
    rsx, rsxy = packed_oracle_sums(S, S2)
    assert np.array_equal(sx, rsx)
    assert np.array_equal(sxy, rsxy)
    assert (cnt == L).all()


SHAPES = [
    (2, 1, 1), (2, 63, 33), (3, 64, 2), (3, 65, 3), (7, 1, 512), (7, 65, 31),
    (15, 64, 64), (16, 17, 40), (19, 1, 1), (19, 63, 512), (19, 65, 33), (20, 64, 7),
    (31, 64, 96), (32, 33, 64), (36, 65, 65), (47, 16, 32), (48, 63, 100),
    (63, 20, 37), (64, 17, 64), (72, 65, 33), (79, 9, 40),
]


@pytest.mark.parametrize("nbeam,nchan,L", SHAPES)
def test_ccm_shapes_bit_exact(dev, nbeam, nchan, L):
    rng = np.random.default_rng(nbeam * 1000 + nchan * 10 + L)
    nsub = 3
    x = rng.integers(0, 256, size=(nbeam, nsub * L + 5, nchan), dtype=np.uint8)
    x[:, :L // 2 + 1, :] = rng.choice([0, 255], size=(nbeam, L // 2 + 1, nchan)).astype(np.uint8)
    S, S2 = ccm.sums_int64(x, L, nsub, t0=2)
    rsx, rsxy = packed_oracle_sums(S, S2)
    variants = [1, 2] if nbeam <= 20 else [1]
    for v in variants:
        say("ccm shape", nbeam, nchan, L, "variant", v)
        sx, sxy, cnt, _ = run_ccm(x, L, nsub, dev, v, t0=2)
        assert np.array_equal(sx, rsx), (nbeam, nchan, L, v)
        assert np.array_equal(sxy, rsxy), (nbeam, nchan, L, v)


def test_ccm_accumulate_across_calls(dev):
    import torch
    from paper_2512_16278_amd import rfi
    rng = np.random.default_rng(5)
    nb, nc, L, nsub = 19, 70, 100, 2
    x = rng.integers(0, 256, size=(nb, 2 * nsub * L, nc), dtype=np.uint8)
    buf = upload(x, dev)
    blk = rfi.make_block(buf, nc)
    sx, sxy, cnt = sums_buffers(nb, nsub, nc, dev)
    say("ccm accumulate")
    rfi.rfi_ccm_accumulate(blk, 0, L, nsub, sx, sxy, cnt, accumulate=0)
    rfi.rfi_ccm_accumulate(blk, nsub * L, L, nsub, sx, sxy, cnt, accumulate=1)
    torch.cuda.synchronize()
    S1, S21 = ccm.sums_int64(x, L, nsub, 0)
    S2_, S22 = ccm.sums_int64(x, L, nsub, nsub * L)
    rsx, rsxy = packed_oracle_sums(S1 + S2_, S21 + S22)
    assert np.array_equal(sx.cpu().numpy(), rsx)
    assert np.array_equal(sxy.cpu().numpy(), rsxy)
    assert (cnt.cpu().numpy() == 2 * L).all()


def test_ccm_largest_exact_count(dev):
    # 255^2 * 33025 = 2147450625 < 2^31: the largest sum the int32 path allows
    nb, nc, L = 3, 16, 33025
    x = np.full((nb, L, nc), 255, dtype=np.uint8)
    x[1, ::2, :] = 0
    say("ccm max count")
    sx, sxy, cnt, _ = run_ccm(x, L, 1, dev, 1)
    S, S2 = ccm.sums_int64(x, L, 1)
    rsx, rsxy = packed_oracle_sums(S, S2)
    assert np.array_equal(sx, rsx) and np.array_equal(sxy, rsxy)
    assert sxy.max() == 255 * 255 * 33025


def _eig_case(dev, x, L, nsub, precision=32, solver=0, refine=1):
    import torch
    from paper_2512_16278_amd import rfi
    nb, _, nc = x.shape
    _, _, _, (buf, blk, sx, sxy, cnt) = run_ccm(x, L, nsub, dev, 1)
    stat, status, ev, v1 = eig_buffers(nb, nsub * nc, dev)
    say("eig", nb, nc, L, "precision", precision, "solver", solver)
    rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, eigvals=ev, v1=v1,
                        precision=precision, solver=solver, refine=refine)
    torch.cuda.synchronize()
    return (stat.cpu().numpy(), status.cpu().numpy(), ev.cpu().numpy(), v1.cpu().numpy())


def _check_eig(x, L, nsub, out, lam_tol, stat_tol):
    stat, status, ev, v1 = out
    cr = pipeline.cells(x, L, nsub)
    nb = x.shape[0]
    ncell = cr.stat.size
    w = cr.w.reshape(ncell, nb)
    lam1 = np.abs(w[:, 0])
    err = np.abs(ev.T - w).max(axis=1) / lam1
    assert err.max() <= lam_tol, err.max()
    ds = np.abs(stat - cr.stat.ravel())
    assert ds.max() <= stat_tol, ds.max()
    # eigenvector: residual against the FP64 matrix, and agreement where the gap is clear
    r = cr.r.reshape(ncell, nb, nb)
    res = np.linalg.norm(np.einsum("cab,bc->ac", r, v1.astype(np.float64)) -
                         w[:, 0][None, :] * v1, axis=0)
    assert res.max() < 5e-4 * lam1.max(), res.max()
    gap = (w[:, 0] - w[:, 1]) / lam1
    clear = gap > 0.05
    vo = cr.v1.reshape(ncell, nb)
    # the sign convention (sum > 0) is decided by rounding when sum(v1) ~ 0:
    # there either sign is valid and the comparison is up to sign
    tie = np.abs(vo.sum(axis=1)) < 1e-5
    d_same = np.abs(v1.T - vo).max(axis=1)
    d_flip = np.abs(v1.T + vo).max(axis=1)
    d = np.where(tie, np.minimum(d_same, d_flip), d_same)
    assert d[clear].max() < 1e-4
    assert np.allclose(np.linalg.norm(v1, axis=0), 1.0, atol=1e-5)
    return status, cr


def test_eig_lane_tiny(dev, tiny):
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    out = _eig_case(dev, x, L, nsub, 32, 1)
    status, cr = _check_eig(x, L, nsub, out, 1e-5, 1e-9)
    assert (status == 0).all()


@pytest.mark.parametrize("solver", [1, 4])
@pytest.mark.parametrize("nbeam", [2, 3, 5, 7, 8, 11, 12, 14, 16, 17, 18, 19, 20])
def test_eig_lane_sizes(dev, nbeam, solver):
    """Per-lane solvers (1: Jacobi, 4: Householder + Sturm), FP32 with the FP64
    refinement: eigenvalues within 1e-5 of lambda_1, statistic within 1e-9.
    Beam counts below their kernel instance (11 in 12, 14 in 16, 17 and 18 in
    20) exercise the padding: clamped rows of the sums and the Sturm count
    with padding selects."""
    rng = np.random.default_rng(100 + nbeam)
    L, nsub, nc = 256, 2, 70
    x = np.clip(np.rint(128 + 20 * rng.standard_normal((nbeam, nsub * L, nc))), 0, 255).astype(np.uint8)
    common = np.rint(15 * np.sin(np.arange(nsub * L) / 5.0)).astype(np.int64)
    x[:, :, 3] = np.clip(x[:, :, 3].astype(np.int64) + common[None, :], 0, 255)
    out = _eig_case(dev, x, L, nsub, 32, solver)
    _check_eig(x, L, nsub, out, 1e-5, 1e-9)


def test_eig_lane_tri_tiny(dev, tiny):
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    out = _eig_case(dev, x, L, nsub, 32, 4)
    status, cr = _check_eig(x, L, nsub, out, 1e-5, 1e-9)
    assert (status == 0).all()


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("nbeam", [2, 7, 19, 36, 72])
def test_eig_wave(dev, nbeam, precision):
    rng = np.random.default_rng(200 + nbeam)
    L, nsub, nc = 128, 2, 9
    x = np.clip(np.rint(128 + 20 * rng.standard_normal((nbeam, nsub * L, nc))), 0, 255).astype(np.uint8)
    common = np.rint(12 * np.sin(np.arange(nsub * L) / 3.0)).astype(np.int64)
    x[:, :, 2] = np.clip(x[:, :, 2].astype(np.int64) + common[None, :], 0, 255)
    out = _eig_case(dev, x, L, nsub, precision, 2)
    tol_l = 1e-5 if precision == 32 else 1e-6
    tol_s = 1e-9 if precision == 32 else 1e-12
    _check_eig(x, L, nsub, out, tol_l, tol_s)


@pytest.mark.parametrize("nbeam", [2, 3, 7, 19, 36, 47, 64, 65, 72, 79])
def test_eig_tridiag(dev, nbeam):
    """Householder-tridiagonal FP64 solver: eigenvalues (FP32 output) within
    1e-6 of lambda_1, statistic within 1e-12, v1 as for the other solvers."""
    rng = np.random.default_rng(400 + nbeam)
    L, nsub, nc = 160, 2, 11
    x = np.clip(np.rint(128 + 20 * rng.standard_normal((nbeam, nsub * L, nc))), 0, 255).astype(np.uint8)
    common = np.rint(12 * np.sin(np.arange(nsub * L) / 3.0)).astype(np.int64)
    x[:, :, 2] = np.clip(x[:, :, 2].astype(np.int64) + common[None, :], 0, 255)
    x[: nbeam // 2, :, 5] = np.clip(x[: nbeam // 2, :, 5].astype(np.int64) + common[None, :], 0, 255)
    out = _eig_case(dev, x, L, nsub, 32, 3)
    status, _ = _check_eig(x, L, nsub, out, 1e-6, 1e-12)
    assert (status == 0).all()


def test_eig_tridiag_72_beams_many_cells(dev):
    """The 72-beam class at the shape the uneven batch runs (L = 512) over
    4200 cells, so that many workgroups and the XCD-contiguous cell order
    are in play: the rows-layout call and the whole-block call (cell-record
    layout) against the oracle, statistic within 1e-12, equal to each other
    bit for bit, masks identical to the oracle's clip."""
    import torch
    from paper_2512_16278_amd import rfi
    rng = np.random.default_rng(472)
    nb, L, nsub, nc = 72, 512, 2, 2100
    x = 128 + 20 * rng.standard_normal((nb, nsub * L, nc))
    t = np.arange(nsub * L)
    for j in rng.choice(nc, size=60, replace=False):          # common-mode RFI channels
        g = rng.uniform(0.3, 2.0, nb)
        x[:, :, j] += 10 * g[:, None] * np.sin(2 * np.pi * t / rng.uniform(20, 200) + j)[None, :]
    x = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    out = _eig_case(dev, x, L, nsub, 32, 3)
    status, cr = _check_eig(x, L, nsub, out, 1e-6, 1e-12)
    assert (status == 0).all()
    buf = upload(x, dev)
    blk = rfi.make_block(buf, nc)
    p = rfi.process_params(L, nsub)
    ws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, p), dtype=torch.uint8, device=dev)
    ncell = nsub * nc
    stat = torch.empty(ncell, dtype=torch.float64, device=dev)
    st2 = torch.empty(ncell, dtype=torch.uint8, device=dev)
    mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
    say("eig 72 beams: whole-block call")
    rfi.rfi_process_block(blk, p, stat, st2, mask, ws)
    torch.cuda.synchronize()
    s_blk = stat.cpu().numpy()
    assert np.array_equal(s_blk, out[0])                      # same arithmetic, either layout
    ref = clip.clip_iterative(cr.stat.ravel(), np.ones(ncell, bool), 3.0, 50)
    assert np.array_equal(mask.cpu().numpy().astype(bool), ref.mask)
    assert ref.nflag > 60 * nsub // 2


def _close_pair_block(seed=91, nb=19, L=1024, nsub=2, nc=16):
    """Two disjoint beam groups carrying two different Walsh sequences (exactly
    orthogonal, zero-mean +-1 patterns over every sub-interval) at amplitude
    100: group A (beams 0-8) without noise, so lambda = 9 exactly; group B
    (beams 9-17) with unit noise, so its eigenvalue sits ~1e-4 below 9; beam
    18 is noise. lambda_1 and lambda_2 are 3e-5 .. 1e-3 apart (relative)."""
    rng = np.random.default_rng(seed)
    t = np.arange(nsub * L) % L
    x = np.empty((nb, nsub * L, nc))
    for j in range(nc):
        w1 = 1 - 2 * (np.array([bin(v).count("1") for v in ((5 + 3 * j) & t)]) & 1)
        w2 = 1 - 2 * (np.array([bin(v).count("1") for v in ((300 + 7 * j) & t)]) & 1)
        for b in range(nb):
            if b < 9:
                x[b, :, j] = 128 + 100 * w1
            elif b < 18:
                x[b, :, j] = 128 + 100 * w2 + rng.standard_normal(nsub * L)
            else:
                x[b, :, j] = 128 + 20 * rng.standard_normal(nsub * L)
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("solver,prec", [(1, 32), (4, 32), (3, 32), (2, 64)])
def test_eig_close_dominant_pair(dev, solver, prec):
    """lambda_1 and lambda_2 3e-5 .. 1e-3 apart (see _close_pair_block): the
    statistic must still match the oracle to 1e-12. One vector of inverse
    iteration shifted ~2e-5 above lambda_1 cannot separate such a pair, and
    its Rayleigh quotient misses lambda_1 by a fraction of the gap."""
    nb, L, nsub = 19, 1024, 2
    x = _close_pair_block()
    cr = pipeline.cells(x, L, nsub)
    w = cr.w.reshape(-1, nb)
    gap = (w[:, 0] - w[:, 1]) / w[:, 0]
    assert gap.max() < 2e-3                       # the pair is close by construction
    stat, status, ev, v1 = _eig_case(dev, x, L, nsub, prec, solver)
    assert np.abs(stat - cr.stat.ravel()).max() <= 1e-12
    assert (status & 8 == 0).all()                # refinement succeeded


def test_eig_degenerate_cells(dev):
    rng = np.random.default_rng(7)
    nb, L, nsub, nc = 19, 64, 2, 20
    x = rng.integers(0, 256, size=(nb, nsub * L, nc), dtype=np.uint8)
    x[4, :L, 5] = 77                 # constant beam in cell (0, 5)
    x[:, L:, 9] = 3                  # every beam constant in cell (1, 9)
    for solver, prec in ((1, 32), (2, 32), (2, 64), (3, 32), (4, 32)):
        stat, status, ev, v1 = _eig_case(dev, x, L, nsub, prec, solver)
        cr = pipeline.cells(x, L, nsub)
        deg = cr.degenerate.ravel()
        assert ((status & 1) != 0).tolist() == deg.tolist()
        assert np.abs(stat - cr.stat.ravel()).max() < 1e-9


def _flag_case(dev, s, status, nsub, nchan, kappa=3.0, max_iter=50, protect=None, state=None,
               own_workspace=True):
    import torch
    from paper_2512_16278_amd import rfi
    ws = None
    if own_workspace:
        ws = torch.empty(rfi.rfi_flag_workspace_size(nsub, nchan), dtype=torch.uint8, device=dev)
    st = torch.from_numpy(s.astype(np.float64)).to(dev)
    stt = torch.from_numpy(status.astype(np.uint8)).to(dev)
    mask = torch.full((nsub * nchan,), 9, dtype=torch.uint8, device=dev)
    out = torch.zeros(48, dtype=torch.uint8, device=dev)
    pr = None if protect is None else torch.from_numpy(protect.astype(np.uint8)).to(dev)
    say("flag", nsub, nchan, kappa, max_iter)
    rfi.rfi_flag(nsub, nchan, st, stt, mask, protect_chan=pr, kappa=kappa, max_iter=max_iter,
                 state=state, out=out, workspace=ws)
    torch.cuda.synchronize()
    return mask.cpu().numpy().astype(bool), rfi.flag_stats_from_bytes(out.cpu().numpy().tobytes())


def _synthetic_stat(rng, n, frac):
    s = 0.075 + 0.002 * rng.standard_normal(n)
    k = int(frac * n)
    idx = rng.choice(n, size=k, replace=False)
    s[idx] += rng.uniform(0.003, 0.6, size=k)
    return np.clip(s, 1 / 19, 1.0)


@pytest.mark.parametrize("seed", range(4))
def test_flag_matches_oracle(dev, seed):
    rng = np.random.default_rng(300 + seed)
    nsub, nchan = 37, 513
    s = _synthetic_stat(rng, nsub * nchan, 0.04)
    status = np.zeros(s.size, np.uint8)
    status[rng.choice(s.size, 50, replace=False)] = 1          # degenerate
    protect = (rng.uniform(size=nchan) < 0.02).astype(np.uint8)
    for kappa, max_iter in ((3.0, 50), (5.0, 50), (2.0, 2)):
        mask, st = _flag_case(dev, s, status, nsub, nchan, kappa, max_iter, protect,
                              own_workspace=kappa != 5.0)
        elig = (status == 0) & ~np.tile(protect.astype(bool), nsub)
        ref = clip.clip_iterative(s, elig, kappa, max_iter)
        assert np.array_equal(mask, ref.mask)
        assert st["iterations"] == ref.iterations and bool(st["converged"]) == ref.converged
        assert st["nflag"] == ref.nflag
        for k in ("mu", "sigma", "thr"):
            assert st[k] == getattr(ref, k), k          # bit-equal: one rounding each


def _same(a, b):
    return a == b or (math.isnan(a) and math.isnan(b))


def test_clip_fit_rounding(dev):
    """The clip's fit, mu = Q1 / (N 2^40) and sigma = sqrt((N Q2 - Q1^2) /
    (N^2 2^80)) each rounded once and thr = mu + kappa sigma, against the same
    arithmetic on Python integers (exact rationals, one rounding each), on
    random moment sums spanning N = 1 .. 2^40 and every exponent the clip
    meets, plus hand-made ties and binade edges."""
    import torch
    from paper_2512_16278_amd import rfi
    rng = np.random.default_rng(77)
    cases = []
    for _ in range(4000):
        N = int(2 ** rng.uniform(0, 40))
        qmax = int(2 ** rng.uniform(1, 41))
        Q1 = int(rng.integers(0, 2 ** 62)) * N % (N * qmax + 1)
        lo = -(-Q1 * Q1 // N)                      # ceil(Q1^2 / N): N Q2 >= Q1^2
        extra = int(2 ** rng.uniform(0, 80)) if rng.uniform() < 0.9 else 0
        cases.append((N, Q1, lo + extra))
    # exact small ratios, power-of-two boundaries, equal values (sigma 0)
    cases += [(1, 0, 0), (1, 1 << 40, 1 << 80), (3, 1, 1), (2, 3, 5), (7, 7 << 39, 7 << 78),
              (1 << 20, (1 << 20) * 12345, (1 << 20) * 12345 ** 2), (5, 2 ** 41 - 1, 2 ** 82),
              (2, 0, 2 ** 81), (2, 0, 2 ** 83), (4, 4 << 38, 2 ** 80 + 8), (3, 2 ** 41 + 1, 2 ** 83)]
    n = len(cases)
    N = torch.tensor([c[0] for c in cases], dtype=torch.int64, device=dev)
    limbs = lambda v: [v & (2 ** 64 - 1), v >> 64]
    as_i64 = lambda a: np.array(a, dtype=np.uint64).view(np.int64)
    Q1 = torch.from_numpy(as_i64([limbs(c[1]) for c in cases])).to(dev)
    Q2 = torch.from_numpy(as_i64([limbs(c[2]) for c in cases])).to(dev)
    mu = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty_like(mu)
    th = torch.empty_like(mu)
    say("clip fit", n)
    for kappa in (3.0, 1.7):
        rfi.rfi_clip_fit(N, Q1, Q2, mu, sg, th, kappa=kappa)
        torch.cuda.synchronize()
        gm, gs, gt = mu.cpu().numpy(), sg.cpu().numpy(), th.cpu().numpy()
        for i, (a, b, c) in enumerate(cases):
            m, s_ = clip.moments_from_sums(a, b, c)
            t = m + kappa * s_
            assert (gm[i], gs[i], gt[i]) == (m, s_, t), (i, a, b, c, kappa)


def test_flag_fallback_and_large_tail(dev):
    """Blocks where the sampled prediction of the final threshold is wrong
    (the sampled cells run higher than the rest, so the exact iteration falls
    below the predicted tail bound and takes its full passes), and where the
    tail is too long for registers: both must equal the oracle exactly."""
    rng = np.random.default_rng(500)
    nsub, nchan = 40, 1500                         # 60000 cells > the 16384-cell sample
    ncell = nsub * nchan
    ns = 16384
    sampled = (np.arange(ns, dtype=np.int64) * ncell) // ns
    s = 0.070 + 0.002 * rng.standard_normal(ncell)
    s[sampled] += 0.02                             # the sample sees a shifted population
    s = np.clip(s, 1 / 19, 1.0)
    status = np.zeros(ncell, np.uint8)
    mask, st = _flag_case(dev, s, status, nsub, nchan)
    ref = clip.clip_iterative(s, status == 0, 3.0, 50)
    assert np.array_equal(mask, ref.mask)
    assert (st["mu"], st["sigma"], st["thr"], st["iterations"]) == \
        (ref.mu, ref.sigma, ref.thr, ref.iterations)
    # a 45 % outlier population: the tail list outgrows the registers
    s = _synthetic_stat(rng, 200000, 0.45)
    mask, st = _flag_case(dev, s, np.zeros(s.size, np.uint8), 100, 2000)
    ref = clip.clip_iterative(s, np.ones(s.size, bool), 3.0, 50)
    assert np.array_equal(mask, ref.mask)
    assert (st["mu"], st["sigma"], st["thr"], st["iterations"], st["nflag"]) == \
        (ref.mu, ref.sigma, ref.thr, ref.iterations, ref.nflag)


def test_flag_edge_cases(dev):
    # nothing eligible; a single cell; all-equal values
    for s, status in ((np.full(10, 0.3), np.ones(10, np.uint8)),
                      (np.array([0.2]), np.zeros(1, np.uint8)),
                      (np.full(64, 0.3), np.zeros(64, np.uint8))):
        mask, st = _flag_case(dev, s, status, 1, s.size)
        ref = clip.clip_iterative(s, status == 0, 3.0)
        assert np.array_equal(mask, ref.mask)
        assert st["iterations"] == ref.iterations and st["nflag"] == ref.nflag
        for k in ("mu", "sigma", "thr"):
            assert _same(st[k], getattr(ref, k)), k
    # an empty block (nsub = 0) runs no fit
    mask, st = _flag_case(dev, np.zeros(0), np.zeros(0, np.uint8), 0, 7)
    assert st["iterations"] == 0 and st["nflag"] == 0


def test_flag_stream_state(dev):
    import torch
    from paper_2512_16278_amd import rfi
    rng = np.random.default_rng(400)
    state = torch.zeros(len(bytes(rfi.rfi_stream_state())), dtype=torch.uint8, device=dev)
    ost = clip.StreamState()
    for i in range(3):
        nsub, nchan = 5 + i, 300
        s = _synthetic_stat(rng, nsub * nchan, 0.03 * (i + 1))
        status = np.zeros(s.size, np.uint8)
        mask, st = _flag_case(dev, s, status, nsub, nchan, state=state)
        ref = clip.clip_stream(ost, s, status == 0)
        assert np.array_equal(mask, ref.mask), i
        assert (st["mu"], st["sigma"], st["thr"]) == (ref.mu, ref.sigma, ref.thr), i
    gs = rfi.stream_state_from_bytes(state.cpu().numpy().tobytes())
    assert gs.n == ost.N and gs.nblocks == 3
    assert gs.q1[0] + (gs.q1[1] << 64) == ost.Q1
    assert gs.q2[0] + (gs.q2[1] << 64) == ost.Q2
    for i in range(3):
        h = gs.hist[i]
        assert (h.mu, h.sigma, h.thr, h.iterations) == tuple(ost.history[i]), i


def test_pipeline_tiny_end_to_end(dev, tiny):
    import torch
    from paper_2512_16278_amd import rfi
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    nb, _, nc = x.shape
    _, _, _, (buf, blk, sx, sxy, cnt) = run_ccm(x, L, nsub, dev, 1)
    stat, status, ev, v1 = eig_buffers(nb, nsub * nc, dev)
    mask = torch.empty(nsub * nc, dtype=torch.uint8, device=dev)
    bmask = torch.empty((nb, nsub * nc), dtype=torch.uint8, device=dev)
    say("pipeline tiny")
    rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, v1=v1)
    rfi.rfi_flag(nsub, nc, stat, status, mask)
    rfi.rfi_eigvec_flag(nb, nsub, nc, v1, mask, status, bmask, kappa_v=1.0)
    torch.cuda.synchronize()
    cr, res, bm = pipeline.block(x, L, nsub, kappa_v=1.0)
    m = mask.cpu().numpy().astype(bool)
    assert np.array_equal(m, res.mask.ravel())
    # injected common-mode cells are flagged; the beam-0 pulse is not a source of flags
    for s_ in spec.sinusoids:
        for k in range(s_.t_lo // L, s_.t_hi // L):
            assert m[k * nc + s_.chan]
    # per-beam stage: identical except where |v| sits within FP32 resolution of the threshold
    g = bmask.cpu().numpy().astype(bool)
    ref = bm.reshape(nb, -1)
    diff = g != ref
    if diff.any():
        _, mu, sd = eigvec.eigvec_mask(cr.v1.reshape(-1, nb), res.mask.ravel(),
                                       np.ones(res.mask.size, bool), 1.0)
        a = np.abs(cr.v1.reshape(-1, nb)).T
        thr = (mu + sd)[:, None]
        assert (np.abs(a - thr)[diff] < 1e-5).all()


def test_synth_gpu_matches_cpu(dev):
    import torch
    from paper_2512_16278_amd import rfi, synth
    for spec, window in ((synth.tiny_spec(), (0, None)),
                         (synth.fast_spec(nchan=4096), (200000, 203450))):
        ds = rfi.DeviceSynth(spec)
        t_lo, t_hi = window
        t_hi = spec.nsamp if t_hi is None else t_hi
        stride = (spec.nchan + 15) // 16 * 16
        for b in (0, spec.nbeam - 1):
            buf = torch.zeros((spec.nsamp, stride), dtype=torch.uint8, device=dev)
            say("synth", spec.name, b)
            ds.fill(buf, b, t_lo, t_hi)
            torch.cuda.synchronize()
            got = buf[t_lo:t_hi, :spec.nchan].cpu().numpy()
            ref = synth.generate(spec, t_lo, t_hi, beams=[b])[0]
            assert np.array_equal(got, ref), (spec.name, b)
