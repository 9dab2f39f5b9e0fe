"""The seeded input generator: known answers and chunk addressability."""
import numpy as np

from paper_2512_16278_amd import synth


def test_philox_known_answers():
    # Philox4x32-10 known-answer vectors (Salmon et al., SC 2011 reference set)
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
        ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
        ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
         (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
    ]
    for ctr, key, out in cases:
        got = synth.philox4x32_10(*[np.array([c]) for c in ctr], *key)
        assert tuple(int(g[0]) for g in got) == out


def test_chunks_regenerate_identically():
    spec = synth.tiny_spec()
    full = synth.generate(spec)
    part = synth.generate(spec, t_lo=1000, t_hi=3100, c_lo=5, c_hi=37, beams=[0, 3, 18])
    assert np.array_equal(part, full[[0, 3, 18], 1000:3100, 5:37])


def test_noise_distribution():
    spec = synth.tiny_spec()
    spec.sinusoids, spec.bursts, spec.pulses = [], [], []
    x = synth.generate(spec, t_hi=2048).astype(np.float64)
    assert abs(x.mean() - 128.0) < 0.1
    assert abs(x.std() - np.sqrt(400 + 1 / 12.0)) < 0.1
    # independent across beams and channels
    c = np.corrcoef(x[:, :, 3])
    assert np.abs(c - np.eye(19)).max() < 0.1


def test_pulse_only_in_its_beam():
    spec = synth.tiny_spec()
    spec.sinusoids, spec.bursts = [], []
    a = synth.generate(spec)
    spec.pulses = []
    b = synth.generate(spec)
    diff = (a != b).any(axis=(1, 2))
    assert diff[0] and not diff[1:].any()


def test_cdf_table_monotone_and_saturated():
    t = synth.normal_cdf_table(10.0)
    assert (np.diff(t.astype(np.int64)) >= 0).all()
    assert t[0] < 100 and t[-1] > 0xFFFFFF00


def test_fast_spec_shapes():
    spec = synth.fast_spec()
    assert spec.nsamp == 203450 and spec.nsamp // spec.L == 99
    assert len(spec.sinusoids) == 82 and len(spec.bursts) == 1
    tabs = synth.device_tables(spec)
    assert tabs["cdf"].shape == (19, 255) and tabs["sin_of_chan"].shape == (4096,)
