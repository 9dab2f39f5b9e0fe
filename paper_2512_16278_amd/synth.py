"""Seeded synthetic multi-beam filterbank data with FAST-like shapes.

This module generates INPUTS only. It holds none of the method's arithmetic
(no sums, correlations, eigenvalues or thresholds), so that the FP64 oracle
and the HIP path can both consume its bytes without sharing code. The bytes
are a pure integer function of (seed, beam, time, channel): any chunk can be
regenerated on its own, on the CPU here or on the GPU by the twin kernel in
``csrc/synth.hip`` (which reads the same integer tables built here).

Sample model, one uint8 total-power value per (beam b, time t, channel c):

    u    = Philox4x32-10(key = seed, counter = (t, c >> 2, b, 0))[c & 3]
    base = #{k in 0..254 : cdf_b[k] <= u}          (discretised N(128, sigma_b))
    v    = base + sinusoids + bursts + pulses       (integers)
    x    = clip(v, 0, 255)

* Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror & Shaw,
  "Parallel random numbers: as easy as 1, 2, 3" (SC 2011).
* cdf_b[k] = round(2^32 * Phi((k + 0.5 - 128) / sigma_b)): inverse-CDF
  sampling of round(128 + sigma_b z) clipped to [0, 255].
* sinusoid i (common to all beams of one channel, over [t_lo, t_hi)):
  (tab_i[(t + phase_i) mod P_i] * gain_ib + 2^15) >> 16 with tab = round(256 A
  sin(2 pi p / P)), gain = round(256 g_b): narrow-band RFI seen by every beam.
* burst i: + amp_ib for t in [t_lo, t_hi), every channel: broadband RFI.
* pulse i (one beam only): + amp when d = t - t0_i - delay_ic >= 0 and
  d mod period_i < width_i, with the cold-plasma delay
  4.148808e3 s MHz^2 cm^3 / pc * DM * (f_c^-2 - f_top^-2): a dispersed
  single-beam astronomical pulse, the negative control.

The observation shapes follow the paper's FAST data (Sec. 2): 19 beams,
4096 x 122.07 kHz channels over 1000-1500 MHz, 49.152 us samples, 8 bits.
Amplitudes, periods and positions of the injected signals are builder
choices; the paper gives none.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TSAMP = 49.152e-6
F_LO, F_HI = 1000.0, 1500.0
KDM = 4.148808e3            # s MHz^2 cm^3 pc^-1
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on uint64 NumPy arrays holding 32-bit words.

    Returns the four 32-bit output words (as uint64 arrays)."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    s32 = np.uint64(32)
    m32 = np.uint64(MASK32)
    for _ in range(10):
        p0 = c0 * m0
        p1 = c2 * m1
        hi0, lo0 = p0 >> s32, p0 & m32
        hi1, lo1 = p1 >> s32, p1 & m32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return c0, c1, c2, c3


def normal_cdf_table(sigma: float, mean: float = 128.0) -> np.ndarray:
    """cdf[k] = round(2^32 Phi((k + 0.5 - mean) / sigma)), k = 0..254, as
    uint32 (saturated at 2^32 - 1)."""
    k = np.arange(255, dtype=np.float64)
    z = (k + 0.5 - mean) / sigma
    phi = np.array([0.5 * math.erfc(-v / math.sqrt(2.0)) for v in z])
    t = np.rint(phi * 4294967296.0)
    return np.minimum(t, 4294967295.0).astype(np.uint32)


@dataclass
class Sinusoid:
    chan: int
    t_lo: int
    t_hi: int
    period: int
    phase: int
    tab: np.ndarray          # int32 [period]
    gain: np.ndarray         # int32 [nbeam]


@dataclass
class Burst:
    t_lo: int
    t_hi: int
    amp: np.ndarray          # int32 [nbeam]


@dataclass
class Pulse:
    beam: int
    t0: int
    period: int
    width: int
    amp: int
    delay: np.ndarray        # int32 [nchan]
    dm: float = 0.0


@dataclass
class SynthSpec:
    nbeam: int
    nchan: int
    nsamp: int
    seed: int
    sigma: np.ndarray                       # float [nbeam]
    sinusoids: list = field(default_factory=list)
    bursts: list = field(default_factory=list)
    pulses: list = field(default_factory=list)
    L: int = 0                              # intended sub-interval length
    name: str = ""

    @property
    def key(self):
        return self.seed & MASK32, (self.seed >> 32) & MASK32

    def cdf_tables(self) -> np.ndarray:
        return np.stack([normal_cdf_table(float(s)) for s in self.sigma])

    def nbytes(self) -> int:
        return self.nbeam * self.nsamp * self.nchan


def generate(spec: SynthSpec, t_lo: int = 0, t_hi: int | None = None,
             c_lo: int = 0, c_hi: int | None = None, beams=None) -> np.ndarray:
    """Bytes x[beam, t, c] for t in [t_lo, t_hi), c in [c_lo, c_hi)."""
    t_hi = spec.nsamp if t_hi is None else t_hi
    c_hi = spec.nchan if c_hi is None else c_hi
    beams = list(range(spec.nbeam)) if beams is None else list(beams)
    nt, nc = t_hi - t_lo, c_hi - c_lo
    cdf = spec.cdf_tables()
    k0, k1 = spec.key
    t = np.arange(t_lo, t_hi, dtype=np.int64)[:, None]
    c = np.arange(c_lo, c_hi, dtype=np.int64)[None, :]
    out = np.empty((len(beams), nt, nc), dtype=np.uint8)
    # Philox blocks cover 4 channels; evaluate the blocks that touch [c_lo, c_hi)
    g_lo, g_hi = c_lo >> 2, (c_hi + 3) >> 2
    g = np.arange(g_lo, g_hi, dtype=np.int64)[None, :]
    tt = np.broadcast_to(t, (nt, g_hi - g_lo))
    gg = np.broadcast_to(g, (nt, g_hi - g_lo))
    sel_word = (c & 3)
    sel_blk = (c >> 2) - g_lo
    for i, b in enumerate(beams):
        w = philox4x32_10(tt, gg, np.full_like(tt, b), np.zeros_like(tt), k0, k1)
        words = np.stack(w, axis=-1)                           # [nt, ng, 4]
        u = words[:, sel_blk[0], sel_word[0]].astype(np.uint32)  # [nt, nc]
        v = np.searchsorted(cdf[b], u, side="right").astype(np.int64)
        for s in spec.sinusoids:
            if not (c_lo <= s.chan < c_hi):
                continue
            a, z = max(t_lo, s.t_lo), min(t_hi, s.t_hi)
            if a >= z:
                continue
            ts = np.arange(a, z, dtype=np.int64)
            val = (s.tab[(ts + s.phase) % s.period].astype(np.int64) * int(s.gain[b]) + (1 << 15)) >> 16
            v[a - t_lo:z - t_lo, s.chan - c_lo] += val
        for bu in spec.bursts:
            a, z = max(t_lo, bu.t_lo), min(t_hi, bu.t_hi)
            if a < z:
                v[a - t_lo:z - t_lo, :] += int(bu.amp[b])
        for p in spec.pulses:
            if p.beam != b:
                continue
            d = t - p.t0 - p.delay[None, c_lo:c_hi].astype(np.int64)
            on = (d >= 0) & ((d % p.period) < p.width)
            v += on * p.amp
        out[i] = np.clip(v, 0, 255).astype(np.uint8)
    return out


def chan_freqs(nchan: int) -> np.ndarray:
    """Channel centre frequencies (MHz) over 1000-1500 MHz (Sec. 2)."""
    return F_LO + (np.arange(nchan) + 0.5) * (F_HI - F_LO) / nchan


def dispersion_delay_samples(nchan: int, dm: float) -> np.ndarray:
    """Cold-plasma delay relative to the top of the band, in samples."""
    f = chan_freqs(nchan)
    d = KDM * dm * (f ** -2.0 - F_HI ** -2.0) / TSAMP
    return np.rint(d).astype(np.int32)


def _sin_table(amp: float, period: int) -> np.ndarray:
    p = np.arange(period, dtype=np.float64)
    return np.rint(256.0 * amp * np.sin(2.0 * np.pi * p / period)).astype(np.int32)


def _gains(rng, nbeam, lo, hi) -> np.ndarray:
    return np.rint(256.0 * rng.uniform(lo, hi, size=nbeam)).astype(np.int32)


def tiny_spec(seed: int = 20251216, nbeam: int = 19, nchan: int = 64, nsub: int = 16,
              L: int = 1024) -> SynthSpec:
    """Small plain-method case: 19 beams x 64 channels x 16 sub-ints x 1024.

    Noise N(128, 20). Narrow-band sinusoid common to all beams (gains
    U(0.5, 1.5), A = 10, P = 64) in 4 channels over 3 consecutive sub-ints;
    one broadband impulse (8 samples, all channels, amplitude 60 U(0.5, 1.5))
    in one sub-int; a periodic dispersed pulse in beam 0 only (period 333,
    width 4, amplitude 40), which must stay unflagged.
    """
    rng = np.random.default_rng(seed)
    nsamp = nsub * L
    spec = SynthSpec(nbeam, nchan, nsamp, seed, np.full(nbeam, 20.0), L=L, name="tiny")
    chans = rng.choice(nchan, size=4, replace=False)
    k0 = int(rng.integers(0, nsub - 3))
    for ch in chans:
        spec.sinusoids.append(Sinusoid(int(ch), k0 * L, (k0 + 3) * L, 64,
                                       int(rng.integers(0, 64)), _sin_table(10.0, 64),
                                       _gains(rng, nbeam, 0.5, 1.5)))
    kb = int(rng.integers(0, nsub))
    tb = kb * L + int(rng.integers(0, L - 8))
    amp = np.rint(60.0 * rng.uniform(0.5, 1.5, size=nbeam)).astype(np.int32)
    spec.bursts.append(Burst(tb, tb + 8, amp))
    spec.pulses.append(Pulse(0, int(rng.integers(0, 333)), 333, 4, 40,
                             dispersion_delay_samples(nchan, 5.0), dm=5.0))
    return spec


def fast_spec(seed: int = 20251217, nbeam: int = 19, nchan: int = 4096,
              seconds: float = 10.0, L: int = 2048, sigma=None,
              frac_chan: float = 0.02, frac_sub: float = 0.005,
              n_pulse_beams: int = 3) -> SynthSpec:
    """FAST-shaped block: 19 beams x 4096 channels, 49.152 us, 10 s.

    Noise N(128, sigma_b) (sigma_b = 20 unless given). ceil(2% of channels)
    carry persistent common-mode sinusoids (A = 8, gains U(0.3, 2), periods
    32..512 samples, random phases); ceil(0.5% of sub-ints) carry a broadband
    burst (64 samples, amplitude 40 U(0.3, 2)); single-beam dispersed pulses
    (DM 50..300, periods 0.3..1.5 s, width 8, amplitude 30) in a few beams.
    """
    rng = np.random.default_rng(seed)
    nsamp = int(seconds / TSAMP)          # whole samples within the duration
    nsub = nsamp // L
    sig = np.full(nbeam, 20.0) if sigma is None else np.asarray(sigma, dtype=np.float64)
    spec = SynthSpec(nbeam, nchan, nsamp, seed, sig, L=L, name="fast")
    n_rfi = int(math.ceil(frac_chan * nchan))
    for ch in rng.choice(nchan, size=n_rfi, replace=False):
        P = int(rng.integers(32, 513))
        spec.sinusoids.append(Sinusoid(int(ch), 0, nsamp, P, int(rng.integers(0, P)),
                                       _sin_table(8.0, P), _gains(rng, nbeam, 0.3, 2.0)))
    n_burst = int(math.ceil(frac_sub * max(nsub, 1)))
    for kb in rng.choice(max(nsub, 1), size=n_burst, replace=False):
        tb = int(kb) * L + int(rng.integers(0, max(L - 64, 1)))
        amp = np.rint(40.0 * rng.uniform(0.3, 2.0, size=nbeam)).astype(np.int32)
        spec.bursts.append(Burst(tb, tb + 64, amp))
    for b in rng.choice(nbeam, size=min(n_pulse_beams, nbeam), replace=False):
        dm = float(rng.uniform(50.0, 300.0))
        period = int(round(rng.uniform(0.3, 1.5) / TSAMP))
        spec.pulses.append(Pulse(int(b), int(rng.integers(0, period)), period, 8, 30,
                                 dispersion_delay_samples(nchan, dm), dm=dm))
    return spec


def mixed_spec(seed: int, nbeam: int, nchan: int, L: int, seconds: float) -> SynthSpec:
    """One block of the uneven mix (PAF-like beam counts): per-beam
    sigma ~ U(10, 30) and the RFI statistics of ``fast_spec``."""
    rng = np.random.default_rng(seed ^ 0x5EED)
    sig = rng.uniform(10.0, 30.0, size=nbeam)
    return fast_spec(seed=seed, nbeam=nbeam, nchan=nchan, seconds=seconds, L=L, sigma=sig)


# --- flat integer tables for the GPU twin generator --------------------------

def device_tables(spec: SynthSpec) -> dict:
    """All integer tables the GPU generator needs, as flat NumPy arrays."""
    nb, nc = spec.nbeam, spec.nchan
    sin_of_chan = np.full(nc, -1, dtype=np.int32)
    nsin = len(spec.sinusoids)
    pmax = max([s.period for s in spec.sinusoids], default=1)
    sin_meta = np.zeros((max(nsin, 1), 4), dtype=np.int64)   # t_lo, t_hi, period, phase
    sin_tab = np.zeros((max(nsin, 1), pmax), dtype=np.int32)
    sin_gain = np.zeros((max(nsin, 1), nb), dtype=np.int32)
    for i, s in enumerate(spec.sinusoids):
        if sin_of_chan[s.chan] >= 0:
            raise ValueError("at most one sinusoid per channel")
        sin_of_chan[s.chan] = i
        sin_meta[i] = (s.t_lo, s.t_hi, s.period, s.phase)
        sin_tab[i, :s.period] = s.tab
        sin_gain[i] = s.gain
    nbu = len(spec.bursts)
    burst_meta = np.zeros((max(nbu, 1), 2), dtype=np.int64)
    burst_amp = np.zeros((max(nbu, 1), nb), dtype=np.int32)
    for i, bu in enumerate(spec.bursts):
        burst_meta[i] = (bu.t_lo, bu.t_hi)
        burst_amp[i] = bu.amp
    npu = len(spec.pulses)
    pulse_meta = np.zeros((max(npu, 1), 5), dtype=np.int64)   # beam, t0, period, width, amp
    pulse_delay = np.zeros((max(npu, 1), nc), dtype=np.int32)
    for i, p in enumerate(spec.pulses):
        pulse_meta[i] = (p.beam, p.t0, p.period, p.width, p.amp)
        pulse_delay[i] = p.delay
    return dict(cdf=spec.cdf_tables(), sin_of_chan=sin_of_chan, sin_meta=sin_meta,
                sin_tab=sin_tab, sin_gain=sin_gain, pmax=pmax, nsin=nsin,
                burst_meta=burst_meta, burst_amp=burst_amp, nburst=nbu,
                pulse_meta=pulse_meta, pulse_delay=pulse_delay, npulse=npu)
