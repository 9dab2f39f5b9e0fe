"""GPU: the serving session (continuous batching of blocks from many streams).

* Each block's result is the same alone and in the mix: every stream is run
  once through a one-slot session on its own, and once interleaved with the
  other streams through a multi-slot session. Statistic, cell status and mask
  must be bit-identical, and so must the clip summaries.
* Against the oracle: the blocks of a stream are cut at arbitrary sample
  counts, so sub-intervals span block boundaries (the carry). The oracle
  forms the sub-intervals of the concatenated samples, and the cells of block
  i are the sub-intervals that end inside it; the clip is the pooled stream
  clip, block by block. Statistic within 1e-9, masks identical.
* Long sub-intervals (past the int32 bound): the carry in int64 records,
  against the oracle and alone against the mix.
* Export / import: a stream split across two sessions through a checkpoint
  gives the same results as the uninterrupted stream.
* Errors, cancellation, budget.
"""
import numpy as np
import pytest

from gpu_util import say, upload
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
    rng = np.random.default_rng(seed)
    x = 128 + 20 * rng.standard_normal((nbeam, nsamp, nchan))
    t = np.arange(nsamp)
    for j in rng.choice(nchan, size=max(1, nchan // 30), replace=False):
        g = rng.uniform(0.5, 1.5, nbeam)
        x[:, :, j] += 12 * g[:, None] * np.sin(2 * np.pi * t / 29.0 + j)[None, :]
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


# (nbeam, nchan, L, block lengths in samples): lengths that are not multiples
# of L, one shorter than L, so that carries open, extend and complete
STREAMS = [
    (19, 100, 256, [700, 300, 100, 900]),
    (7, 64, 128, [128, 500, 77, 333]),
    (36, 40, 300, [1000, 250, 650]),
    (72, 48, 512, [1500, 700, 100, 1300]),     # the 72-beam class, L >= 512
]


def _blocks(dev, spec, seed):
    nb, nc, L, lens = spec
    x = _data(nb, nc, sum(lens), seed)
    bufs, t = [], 0
    for n in lens:
        bufs.append(upload(x[:, t:t + n, :], dev))
        t += n
    return x, bufs


def _run(sess, sid, bufs, nc):
    from paper_2512_16278_amd import rfi
    tickets = [sess.submit(sid, rfi.make_block(b, nc), tag=i) for i, b in enumerate(bufs)]
    return tickets


def _collect(sess, tickets):
    from paper_2512_16278_amd import rfi
    out = []
    for t in tickets:
        r = sess.wait(t, timeout_us=60_000_000)
        assert r.status == rfi.RFI_OK, r.status
        arrs = rfi.result_arrays(sess, r)
        out.append((r.nsub, r.carried, r.carry_samples, arrs,
                    (r.flag.mu, r.flag.sigma, r.flag.thr, r.flag.iterations, r.flag.nflag)))
        sess.release(t)
    return out


def test_serve_alone_equals_mix_and_oracle(dev):
    from paper_2512_16278_amd import rfi
    data = [_blocks(dev, spec, 50 + i) for i, spec in enumerate(STREAMS)]
    # alone: one stream at a time, one block at a time
    alone = []
    for (nb, nc, L, lens), (x, bufs) in zip(STREAMS, data):
        say("serve: alone", nb, nc, L, lens)
        with rfi.Session(max_inflight=1) as s:
            sid = s.open_stream(nb, nc, L)
            alone.append(_collect(s, _run(s, sid, bufs, nc)))
    # mix: all streams interleaved block by block, several slots
    say("serve: mix")
    with rfi.Session(max_inflight=6) as s:
        sids = [s.open_stream(nb, nc, L) for nb, nc, L, _ in STREAMS]
        tickets = [[] for _ in STREAMS]
        for i in range(max(len(sp[3]) for sp in STREAMS)):
            for j, (spec, (x, bufs)) in enumerate(zip(STREAMS, data)):
                if i < len(bufs):
                    tickets[j].append(s.submit(sids[j], rfi.make_block(bufs[i], spec[1]), tag=i))
        mixed = [_collect(s, tk) for tk in tickets]
    for j in range(len(STREAMS)):
        for a, m in zip(alone[j], mixed[j]):
            assert a[:3] == m[:3], j
            for u, v in zip(a[3], m[3]):
                assert np.array_equal(u, v), j
            assert a[4] == m[4] or (np.isnan(a[4][0]) and np.isnan(m[4][0])), j
    # oracle: sub-intervals of the concatenated samples, pooled clip per block
    for (nb, nc, L, lens), (x, _), res in zip(STREAMS, data, alone):
        ksub = x.shape[1] // L
        cr = pipeline.cells(x, L, ksub)
        st = clip.StreamState()
        sg = clip.StreamState()                     # the oracle's clip on the GPU statistic
        ends = np.cumsum(lens)
        done = 0
        for i, (nsub, carried, carry, (stat, cst, mask), fl) in enumerate(res):
            kend = ends[i] // L                     # sub-intervals complete after block i
            rows = slice(done, kend)
            assert nsub == kend - done, (nb, i)
            assert carry == ends[i] - kend * L, (nb, i)
            if nsub:
                so = cr.stat[rows].ravel()
                assert np.abs(stat - so).max() <= 1e-9, (nb, i)
                ref = clip.clip_stream(st, so, ~cr.degenerate[rows].ravel())
                assert np.array_equal(mask.astype(bool), ref.mask), (nb, i)
                assert fl[3] == ref.iterations and fl[4] == ref.nflag, (nb, i)
                # the pooled clip of the session on its own statistic: bit-equal fits
                rg = clip.clip_stream(sg, stat, (cst & (rfi.RFI_CELL_DEGENERATE |
                                                        rfi.RFI_CELL_BAD_COUNT)) == 0)
                assert np.array_equal(mask.astype(bool), rg.mask), (nb, i)
                assert fl[:4] == (rg.mu, rg.sigma, rg.thr, rg.iterations), (nb, i)
            done = kend


def test_serve_beam_stage(dev):
    """Streams opened with the per-beam stage (Sec. 3.3 last paragraph): each
    block also returns v1 and the per-beam mask. The stat, status and mask
    are those of the same stream without the stage, bit for bit; v1 is unit
    norm on every non-degenerate cell (row 0 of a carried block included);
    the per-beam mask equals rfi_eigvec_flag run on the block's own v1, mask
    and status; results are the same alone and in the mix."""
    import torch
    from paper_2512_16278_amd import rfi
    specs = [STREAMS[0], STREAMS[3]]
    data = [_blocks(dev, spec, 70 + i) for i, spec in enumerate(specs)]

    def run(slots, beams):
        out = []
        with rfi.Session(max_inflight=slots) as s:
            sids = [s.open_stream(nb, nc, L, beam_stage=beams, kappa_v=1.0)
                    for nb, nc, L, _ in specs]
            tk = [[s.submit(sid, rfi.make_block(b, spec[1]), tag=i) for i, b in enumerate(bufs)]
                  for sid, spec, (_, bufs) in zip(sids, specs, data)]
            for spec, ts in zip(specs, tk):
                res = []
                for t in ts:
                    r = s.wait(t, timeout_us=60_000_000)
                    assert r.status == rfi.RFI_OK
                    arr = rfi.result_arrays(s, r)
                    if beams:
                        # outputs exist for blocks with cells (a block that only
                        # extends the carry has none)
                        assert bool(r.v1) == bool(r.beam_mask) == (r.nsub > 0)
                        bm = rfi.result_beams(s, r, spec[0])
                    else:
                        assert not r.v1 and not r.beam_mask
                        with pytest.raises(rfi.RfiError):
                            rfi.result_beams(s, r, spec[0])
                        bm = None
                    res.append((r.nsub, r.carried, arr, bm))
                    s.release(t)
                out.append(res)
        return out

    say("serve: beam stage")
    plain = run(1, False)
    alone = run(1, True)
    mixed = run(4, True)
    for j, spec in enumerate(specs):
        nb, nc = spec[0], spec[1]
        for p, a, m in zip(plain[j], alone[j], mixed[j]):
            assert p[:2] == a[:2] == m[:2]
            for u, v, w in zip(p[2], a[2], m[2]):
                assert np.array_equal(u, v) and np.array_equal(v, w)
            assert np.array_equal(a[3][0], m[3][0]) and np.array_equal(a[3][1], m[3][1])
            nsub = a[0]
            if not nsub:
                continue
            stat, cst, mask = a[2]
            v1, bm = a[3]
            ok = (cst & (rfi.RFI_CELL_DEGENERATE | rfi.RFI_CELL_BAD_COUNT)) == 0
            nrm = np.linalg.norm(v1.astype(np.float64), axis=0)
            assert np.abs(nrm[ok] - 1.0).max() < 1e-5
            # the per-beam stage recomputed on the device from the block's own outputs
            vt = torch.from_numpy(v1).to(dev)
            mt = torch.from_numpy(mask).to(dev)
            ct = torch.from_numpy(cst).to(dev)
            bt = torch.empty((nb, nsub * nc), dtype=torch.uint8, device=dev)
            rfi.rfi_eigvec_flag(nb, nsub, nc, vt, mt, ct, bt, kappa_v=1.0)
            torch.cuda.synchronize()
            assert np.array_equal(bt.cpu().numpy(), bm)
            assert not (bm.astype(bool) & ~mask.astype(bool)[None, :]).any()


def test_serve_long_sub_intervals(dev):
    """A stream whose sub-intervals pass the int32 bound (L = 40,960 samples,
    4 s of FAST sampling): its carry is held as int64 cell records and summed
    by the long route (opened, extended, completed, opened again; a block with
    a full sub-interval between a completed carry and a new one). Results are
    the same alone and beside an ordinary stream; against the oracle the
    statistic is within 1e-12 (FP64 tridiagonal solver) and the pooled clip's
    masks are identical."""
    from paper_2512_16278_amd import rfi
    specs = [(19, 16, 40960, [50000, 30000, 20000, 100000]), STREAMS[1]]
    data = [_blocks(dev, spec, 90 + i) for i, spec in enumerate(specs)]
    say("serve: long sub-intervals alone")
    nb, nc, L, lens = specs[0]
    with rfi.Session(max_inflight=1) as s:
        sid = s.open_stream(nb, nc, L)
        alone = _collect(s, _run(s, sid, data[0][1], nc))
    say("serve: long sub-intervals in a mix")
    with rfi.Session(max_inflight=3) as s:
        sids = [s.open_stream(b, c, l) for b, c, l, _ in specs]
        tickets = [[] for _ in specs]
        for i in range(max(len(sp[3]) for sp in specs)):
            for j, (spec, (_, bufs)) in enumerate(zip(specs, data)):
                if i < len(bufs):
                    tickets[j].append(s.submit(sids[j], rfi.make_block(bufs[i], spec[1]), tag=i))
        mixed = [_collect(s, tk) for tk in tickets]
    for a, m in zip(alone, mixed[0]):
        assert a[:3] == m[:3]
        for u, v in zip(a[3], m[3]):
            assert np.array_equal(u, v)
        assert a[4] == m[4] or (np.isnan(a[4][0]) and np.isnan(m[4][0]))
    x = data[0][0]
    ksub = x.shape[1] // L
    say("serve: long sub-intervals, oracle")
    cr = pipeline.cells(x, L, ksub)
    st = clip.StreamState()
    ends = np.cumsum(lens)
    done = 0
    assert [r[1] for r in alone] == [0, 0, 1, 1]           # carries completed
    for i, (nsub, carried, carry, (stat, cst, mask), fl) in enumerate(alone):
        kend = ends[i] // L
        assert nsub == kend - done and carry == ends[i] - kend * L, i
        if nsub:
            rows = slice(done, kend)
            so = cr.stat[rows].ravel()
            assert (cst == 0).all(), i
            assert np.abs(stat - so).max() <= 1e-12, i
            ref = clip.clip_stream(st, so, ~cr.degenerate[rows].ravel())
            assert np.array_equal(mask.astype(bool), ref.mask), i
            assert fl[3] == ref.iterations and fl[4] == ref.nflag, i
        done = kend
    assert done == ksub


def test_serve_export_import(dev):
    from paper_2512_16278_amd import rfi
    nb, nc, L, lens = STREAMS[0]
    x, bufs = _blocks(dev, STREAMS[0], 77)
    say("serve: uninterrupted")
    with rfi.Session(max_inflight=2) as s:
        sid = s.open_stream(nb, nc, L)
        whole = _collect(s, _run(s, sid, bufs, nc))
    say("serve: split at a checkpoint")
    with rfi.Session(max_inflight=2) as s:
        sid = s.open_stream(nb, nc, L)
        first = _collect(s, _run(s, sid, bufs[:2], nc))
        ckpt = s.export_stream(sid)
    with rfi.Session(max_inflight=3) as s:
        sid = s.open_stream(nb, nc, L)
        s.import_stream(sid, ckpt)
        second = _collect(s, _run(s, sid, bufs[2:], nc))
    for a, b in zip(whole, first + second):
        assert a[:3] == b[:3]
        for u, v in zip(a[3], b[3]):
            assert np.array_equal(u, v)


def test_serve_errors_cancel_budget(dev):
    import torch
    from paper_2512_16278_amd import rfi
    nb, nc, L = 19, 64, 128
    x = _data(nb, nc, 40 * L, 5)
    buf = upload(x, dev)
    with rfi.Session(max_inflight=1, hbm_budget=1 << 20) as s:
        sid = s.open_stream(nb, nc, L)
        with pytest.raises(rfi.RfiError) as e:          # the block alone exceeds the budget
            s.submit(sid, rfi.make_block(buf, nc))
        assert e.value.code == rfi.RFI_E_BUDGET
        with pytest.raises(rfi.RfiError):               # shape differs from the stream
            s.submit(sid, rfi.make_block(buf[:7], nc))
        with pytest.raises(rfi.RfiError):
            s.submit(sid + 99, rfi.make_block(buf[:, :L], nc))
        with pytest.raises(rfi.RfiError):
            s.open_stream(nb, nc, 0)
    with rfi.Session(max_inflight=1) as s:
        sid = s.open_stream(nb, nc, L)
        big = s.submit(sid, rfi.make_block(buf, nc))
        small = [s.submit(sid, rfi.make_block(buf[:, :L], nc)) for _ in range(4)]
        code = s.cancel(small[-1])
        r_big = s.wait(big)
        assert r_big.status == rfi.RFI_OK and r_big.nsub == 40
        rs = [s.wait(t) for t in small]
        if code == rfi.RFI_OK:
            assert rs[-1].status == rfi.RFI_E_CANCELLED
        else:
            assert code == rfi.RFI_E_NOT_READY
        for r in rs[:-1]:
            assert r.status == rfi.RFI_OK and r.nsub == 1
        assert s.poll(big) is not None
        s.release(big)
        with pytest.raises(rfi.RfiError):
            s.release(big)                               # already released
        with pytest.raises(rfi.RfiError):
            s.wait(big)
        # a block shorter than L only extends the carry: no cells
        sid2 = s.open_stream(nb, nc, L)
        r = s.wait(s.submit(sid2, rfi.make_block(buf[:, :L // 2], nc)))
        assert r.status == rfi.RFI_OK and r.nsub == 0 and r.carry_samples == L // 2
        r = s.wait(s.submit(sid2, rfi.make_block(buf[:, :L // 2], nc)))
        assert r.nsub == 1 and r.carried == 1 and r.carry_samples == 0
        s.close_stream(sid2)
        torch.cuda.synchronize()


def _entry(lo, hi, tile=0, stages=0, group=0, solver=0, wg=0):
    from paper_2512_16278_amd import rfi
    return rfi.rfi_tune_entry(lo, hi, tile, stages, group, solver, wg, 0, 0.0, 0.0)


def test_serve_tune_table(dev):
    """A session given a tune table runs every stream with its entry's launch
    choices: tile, ring depth and XCD grouping of the sums are bit-exact with
    the defaults; another solver gives identical masks and statistics within
    the two solvers' accuracies: up to 20 beams the per-lane Jacobi (within
    about 3e-14 of FP64) against the default per-lane Householder, whose Ritz
    subspace carries the rounding of its FP32 reduction (within 3e-12 of
    FP64), so 1e-11; above, 1e-10 for the FP32 wave Jacobi, whose lambda_1 is
    the FP64 Rayleigh quotient of its FP32 vector, error quadratic in that
    vector's. Entries outside the allowed ranges fail rfi_stream_open."""
    from paper_2512_16278_amd import rfi
    t = rfi.rfi_tune_table()
    ents = [_entry(2, 15, stages=2, group=512, solver=rfi.RFI_EIG_LANE, wg=64),
            _entry(16, 31, tile=2, stages=3, group=4096, solver=rfi.RFI_EIG_LANE_TRI, wg=128),
            _entry(32, 47, group=256, solver=rfi.RFI_EIG_WAVE)]
    t.n = len(ents)
    for i, e in enumerate(ents):
        t.e[i] = e
    data = [_blocks(dev, spec, 80 + i) for i, spec in enumerate(STREAMS)]
    res = []
    for table in (None, t):
        say("serve: tune table", table is not None)
        with rfi.Session(max_inflight=4, tune=table) as s:
            sids = [s.open_stream(nb, nc, L) for nb, nc, L, _ in STREAMS]
            tickets = [_run(s, sid, bufs, spec[1])
                       for sid, spec, (x, bufs) in zip(sids, STREAMS, data)]
            res.append([_collect(s, tk) for tk in tickets])
    for j, (nb, nc, L, _) in enumerate(STREAMS):
        # LANE_TRI is the default for 16-31 beams; above 47 the table has no entry
        same_solver = (16 <= nb <= 31) or nb > 47
        for a, m in zip(res[0][j], res[1][j]):
            assert a[:3] == m[:3], nb
            sa, sm = a[3][0], m[3][0]
            if same_solver or sa.size == 0:
                assert np.array_equal(sa, sm), nb
            else:
                assert np.abs(sa - sm).max() <= (1e-11 if nb <= 20 else 1e-10), nb
            assert np.array_equal(a[3][1], m[3][1]), nb
            assert np.array_equal(a[3][2], m[3][2]), nb
    # out-of-range entries are rejected when a stream of that shape opens
    for bad in (_entry(2, 79, tile=1), _entry(2, 79, wg=96), _entry(2, 79, stages=5),
                _entry(2, 79, solver=rfi.RFI_EIG_LANE)):
        tb = rfi.rfi_tune_table()
        tb.n = 1
        tb.e[0] = bad
        with rfi.Session(max_inflight=1, tune=tb) as s:
            with pytest.raises(rfi.RfiError) as ei:
                s.open_stream(36, 40, 300)
            assert ei.value.code == rfi.RFI_E_INVALID
