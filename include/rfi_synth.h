/*
 * rfi_synth.h -- seeded synthetic multi-beam filterbank generator on the GPU
 * (test and benchmark input infrastructure; not part of the method).
 *
 * Produces the same bytes as paper_2512_16278_amd/synth.py: one uint8
 * total-power sample per (beam, time, channel) from Philox4x32-10 keyed by
 * the seed, an inverse-CDF table per beam, and integer tables of injected
 * common-mode sinusoids, broadband bursts and single-beam dispersed pulses.
 * Every pointer in rfi_synth_spec is a DEVICE pointer owned by the caller.
 */
#ifndef RFI_SYNTH_H
#define RFI_SYNTH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nbeam, nchan;
  int64_t nsamp;
  int64_t row_stride;          /* bytes per time row of the destination, multiple of 4 */
  uint32_t key0, key1;         /* Philox key (low, high 32 bits of the seed) */
  const uint32_t* cdf;         /* [nbeam][255] inverse-CDF thresholds */
  const int32_t* sin_of_chan;  /* [nchan] sinusoid index or -1 */
  const int64_t* sin_meta;     /* [nsin][4]: t_lo, t_hi, period, phase */
  const int32_t* sin_tab;      /* [nsin][pmax]: round(256 A sin(2 pi p / P)) */
  const int32_t* sin_gain;     /* [nsin][nbeam]: round(256 g_b) */
  int32_t pmax;
  int32_t nburst;
  const int64_t* burst_meta;   /* [nburst][2]: t_lo, t_hi */
  const int32_t* burst_amp;    /* [nburst][nbeam] */
  int32_t npulse;
  const int64_t* pulse_meta;   /* [npulse][5]: beam, t0, period, width, amp */
  const int32_t* pulse_delay;  /* [npulse][nchan] delay in samples */
} rfi_synth_spec;

/* Fill rows [t_lo, t_hi) of one beam into dst ([t_hi - t_lo][row_stride]
 * bytes, device). Channels >= nchan of each row are left untouched (except
 * inside the last 4-byte group). Returns 0, or -1 for bad arguments, -5 for a
 * launch error. Asynchronous on stream (a hipStream_t). */
int32_t rfi_synth_fill(const rfi_synth_spec* spec, int32_t beam, int64_t t_lo, int64_t t_hi,
                       uint8_t* dst, void* stream);

/* Streaming-read reference for the HBM roofline (measurement infrastructure,
 * not part of the method): reads nbytes of device memory at src once, in
 * 16-byte loads spread over the whole chip, and writes one 32-bit XOR of the
 * data per thread into sink (device, at least rfi_stream_read_sink_words()
 * words) so that the loads cannot be dropped. src 16-byte aligned; nbytes a
 * multiple of 16. Returns 0, -1 for bad arguments, -5 for a launch error.
 * Asynchronous on stream (a hipStream_t). */
int32_t rfi_stream_read_sink_words(void);
int32_t rfi_stream_read(const void* src, int64_t nbytes, uint32_t* sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RFI_SYNTH_H */
