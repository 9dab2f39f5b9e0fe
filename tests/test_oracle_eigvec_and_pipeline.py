"""Pins for oracle/eigvec.py (Sec. 3.3 last paragraph, Sec. 4.5) and
behavioural checks of the composed oracle path on synthetic data."""
import numpy as np
import pytest

from oracle import ccm, clip, eig, eigvec, pipeline
from paper_2512_16278_amd import synth


def test_eigvec_mask_hand_example():
    # 6 cells x 2 beams; cells 4, 5 flagged by the eigenvalue stage
    v1 = np.array([[0.7, 0.7], [0.6, 0.8], [0.8, 0.6], [0.7, 0.7],
                   [0.99, 0.1], [0.1, 0.99]])
    mask = np.array([False, False, False, False, True, True])
    ok = np.ones(6, bool)
    bm, mu, sd = eigvec.eigvec_mask(v1, mask, ok, kappa_v=1.0)
    # clean cells 0..3: beam 0 |v| = .7 .6 .8 .7 -> mu .7, sd sqrt(.005)
    assert abs(mu[0] - 0.7) < 1e-15 and abs(sd[0] - np.sqrt(0.005)) < 1e-15
    assert abs(mu[1] - 0.7) < 1e-15
    thr = 0.7 + np.sqrt(0.005)
    assert bm[0].tolist() == [False] * 4 + [0.99 > thr, 0.1 > thr]
    assert bm[1].tolist() == [False] * 4 + [0.1 > thr, 0.99 > thr]
    assert bm[0, 4] and not bm[0, 5] and bm[1, 5] and not bm[1, 4]


def test_eigvec_mask_uses_magnitudes_and_kappa():
    rng = np.random.default_rng(40)
    v1 = rng.standard_normal((500, 5)) * 0.1 + 0.4
    v1[::7] *= -1
    mask = rng.uniform(size=500) < 0.2
    ok = np.ones(500, bool)
    b1, mu, sd = eigvec.eigvec_mask(v1, mask, ok, 1.0)
    b3, _, _ = eigvec.eigvec_mask(v1, mask, ok, 3.0)
    assert not (b1 & ~mask[None]).any()
    assert (b1 | ~b3).all() and b3.sum() <= b1.sum()
    np.testing.assert_allclose(mu, np.abs(v1[~mask]).mean(0), rtol=1e-14)


@pytest.fixture(scope="module")
def tiny():
    spec = synth.tiny_spec()
    x = synth.generate(spec)
    return spec, x


def test_pipeline_flags_injected_rfi_and_keeps_pulse(tiny):
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    cr, res, _ = pipeline.block(x, L, nsub, kappa=3.0)
    # every cell with the common-mode sinusoid is flagged
    for s in spec.sinusoids:
        for k in range(s.t_lo // L, s.t_hi // L):
            assert res.mask[k, s.chan], (k, s.chan)
    # the broadband burst's sub-int is flagged in most channels
    kb = spec.bursts[0].t_lo // L
    assert res.mask[kb].mean() > 0.9
    assert res.converged


def test_single_beam_pulse_is_a_negative_control(tiny):
    """Differential control: the same bytes with and without the beam-0
    pulse give nearly the same mask (a single-beam signal does not create
    inter-beam correlation)."""
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    spec_np = synth.tiny_spec()
    spec_np.pulses = []
    x_np = synth.generate(spec_np)
    assert (x != x_np).any()
    _, r_p, _ = pipeline.block(x, L, nsub)
    _, r_n, _ = pipeline.block(x_np, L, nsub)
    assert (r_p.mask != r_n.mask).sum() <= 3


def test_protected_channels(tiny):
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    prot = np.zeros(spec.nchan, bool)
    prot[spec.sinusoids[0].chan] = True
    _, res, _ = pipeline.block(x, L, nsub, protect_chan=prot)
    assert not res.mask[:, spec.sinusoids[0].chan].any()


def test_eigvec_stage_on_synthetic(tiny):
    spec, x = tiny
    L, nsub = spec.L, spec.nsamp // spec.L
    cr, res, bm = pipeline.block(x, L, nsub, kappa_v=1.0)
    assert bm.shape == (spec.nbeam, nsub, spec.nchan)
    assert not (bm & ~res.mask[None]).any()
    # kappa_v 1 -> 3 masks fewer beam-cells (Sec. 4.5 trend)
    _, _, bm3 = pipeline.block(x, L, nsub, kappa_v=3.0)
    assert bm3.sum() <= bm.sum()


def test_statistic_on_pure_noise_is_near_marchenko_pastur_edge():
    # sanity: noise-only cells have lambda_1 near (1 + sqrt(n/L))^2
    spec = synth.tiny_spec()
    spec.sinusoids, spec.bursts, spec.pulses = [], [], []
    x = synth.generate(spec, t_lo=0, t_hi=4 * spec.L)
    cr = pipeline.cells(x, spec.L, 4)
    edge = (1 + np.sqrt(spec.nbeam / spec.L)) ** 2
    assert abs(np.median(cr.w[..., 0]) - edge) < 0.1
