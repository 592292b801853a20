/*
 * Seeded synthetic 4+4-bit channelised voltages.
 *
 * This module only makes input bytes. It holds none of the spectral-kurtosis
 * arithmetic (no power, no sums, no normalisation, no estimator): both the
 * CPU oracle and the GPU library consume the bytes it writes.
 *
 * Data model (paper, App. B, digitisation simulation): each complex sample has
 * real and imaginary parts that are Gaussian with RMS sigma_i counts, rounded
 * to the nearest integer and clipped to [-7, 7]. A byte holds one complex
 * sample, offset-encoded: high nibble = Re + 8, low nibble = Im + 8. The byte
 * array is time-major, channels next, inputs innermost: out[t][f][i]
 * (Sec. 3.1: each X-engine node holds time-ordered data for all inputs of a
 * few channels).
 *
 * Randomness comes from one counter-based generator, SplitMix64 (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
 * the n-th output for key k is the SplitMix64 output function applied to
 * k + (n + 1) * 0x9E3779B97F4A7C15. Every sample draws from its own counter,
 * so the bytes do not depend on the number of threads.
 *
 * Outside RFI regions, each component is drawn by inverse CDF against 14
 * per-input integer thresholds (exact and fast). Inside continuous-domain RFI
 * regions (tones, noise bursts, a common-mode signal shared by all inputs)
 * the Gaussian is drawn by Box-Muller in FP64,
 * the interference is added, and the sum is rounded and clipped. Impulsive
 * bursts overwrite samples with a fixed-amplitude phasor.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* n-th output of the SplitMix64 sequence whose state starts at `key`. */
static inline uint64_t syn_draw(uint64_t key, uint64_t n) {
  return splitmix_out(key + (n + 1) * SYN_GAMMA);
}

/* Stream keys: separate sequences for background, noise bursts, phases. */
static uint64_t syn_key(uint64_t seed, uint64_t stream) {
  return splitmix_out(seed * 0xD1B54A32D192ED03ULL + stream * SYN_GAMMA + 1);
}

uint64_t synth_splitmix64(uint64_t key, uint64_t n) { return syn_draw(key, n); }

/* Event kinds. */
enum { SYN_TONE = 1, SYN_NOISE = 2, SYN_BURST = 3, SYN_COMMON = 4 };

typedef struct {
  int32_t kind;
  int32_t channel;
  int64_t t0, t1;     /* [t0, t1) in samples */
  double amplitude;   /* tone/burst amplitude in counts; noise / common-mode RMS per component */
  double nu0, nu1;    /* tone frequency offset (cycles/sample) at t0 and at t1 (linear sweep) */
} syn_event;

typedef struct {
  int32_t n_inputs, n_channels;
  int64_t n_samples;
  uint64_t seed;
  const double* sigma;       /* [N] per-input RMS per component, counts */
  const syn_event* events;   /* [n_events] */
  int32_t n_events;
  int32_t clip;              /* 7 */
} syn_desc;

static double syn_phi(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Thresholds of the rounded, clipped Gaussian: a component equals
 * -clip + #{k : thr[k] <= u} for a 32-bit uniform u. */
void synth_thresholds(double sigma, int clip, uint32_t* thr) {
  for (int k = 0; k < 2 * clip; ++k) {
    double edge = (double)(k - clip) + 0.5;            /* between value k-clip and k-clip+1 */
    double c = syn_phi(edge / sigma);
    double s = floor(c * 4294967296.0);
    if (s < 0) s = 0;
    if (s > 4294967295.0) s = 4294967295.0;
    thr[k] = (uint32_t)s;
  }
}

static inline int syn_clip_round(double x, int clip) {
  double r = floor(x + 0.5);
  if (r > clip) r = clip;
  if (r < -clip) r = -clip;
  return (int)r;
}

static inline uint8_t syn_encode(int re, int im) {
  return (uint8_t)(((re + 8) << 4) | (im + 8));
}

typedef struct {
  const syn_desc* d;
  uint8_t* out;
  const uint32_t* thr;   /* [N][2*clip] */
  const uint8_t* bin;    /* [N][256]: value for top byte of u (bit 7 set: straddles a threshold) */
  int64_t t_begin, t_end;
} syn_job;

/* Component value for uniform u: -clip + #{k : thr[k] <= u}. The per-input
 * table answers directly for the 256-bin of u's top byte unless a threshold
 * falls inside that bin; the result is the same either way. */
static inline int syn_component(uint32_t u, const uint32_t* th, const uint8_t* bin, int C) {
  uint8_t b = bin[u >> 24];
  if (!(b & 0x80)) return (int)b - C;
  int v = -C;
  for (int k = 0; k < 2 * C; ++k) v += (th[k] <= u);
  return v;
}

static void* syn_worker(void* arg) {
  syn_job* j = (syn_job*)arg;
  const syn_desc* d = j->d;
  const int N = d->n_inputs, F = d->n_channels, C = d->clip, NT = 2 * d->clip;
  const uint64_t kbg = syn_key(d->seed, 0), knoise = syn_key(d->seed, 1), kph = syn_key(d->seed, 2);
  const uint64_t kcm = syn_key(d->seed, 4);
  const syn_event* act[64];
  for (int64_t t = j->t_begin; t < j->t_end; ++t) {
    for (int f = 0; f < F; ++f) {
      int na = 0;
      for (int e = 0; e < d->n_events && na < 64; ++e) {
        const syn_event* ev = &d->events[e];
        if (ev->channel == f && t >= ev->t0 && t < ev->t1 && ev->kind != SYN_BURST) act[na++] = ev;
      }
      uint8_t* row = j->out + ((size_t)t * F + f) * N;
      const uint64_t base = ((uint64_t)t * F + f) * (uint64_t)N;
      if (na == 0) {
        for (int i = 0; i < N; ++i) {
          uint64_t r = syn_draw(kbg, base + i);
          uint32_t ure = (uint32_t)(r >> 32), uim = (uint32_t)r;
          const uint32_t* th = j->thr + (size_t)i * NT;
          const uint8_t* bn = j->bin + (size_t)i * 256;
          row[i] = syn_encode(syn_component(ure, th, bn, C), syn_component(uim, th, bn, C));
        }
        continue;
      }
      for (int i = 0; i < N; ++i) {
        uint64_t r = syn_draw(kbg, base + i);
        double u1 = ((double)(r >> 32) + 1.0) / 4294967296.0;   /* (0, 1] */
        double u2 = (double)(uint32_t)r / 4294967296.0;          /* [0, 1) */
        double rad = sqrt(-2.0 * log(u1));
        double xr = d->sigma[i] * rad * cos(2.0 * M_PI * u2);
        double xi = d->sigma[i] * rad * sin(2.0 * M_PI * u2);
        for (int a = 0; a < na; ++a) {
          const syn_event* ev = act[a];
          if (ev->kind == SYN_TONE) {
            double tau = (double)(t - ev->t0);
            double span = (double)(ev->t1 - ev->t0);
            double cyc = ev->nu0 * tau + 0.5 * (ev->nu1 - ev->nu0) * tau * tau / span;
            double ph0 = 2.0 * M_PI * ((double)(syn_draw(kph, (uint64_t)(ev - d->events) * 1000003ULL + i) >> 11) / 9007199254740992.0);
            double th = ph0 + 2.0 * M_PI * (cyc - floor(cyc));
            xr += ev->amplitude * cos(th);
            xi += ev->amplitude * sin(th);
          } else if (ev->kind == SYN_COMMON) {
            /* One Gaussian draw per (t, f), shared by every input (App. A). */
            uint64_t q = syn_draw(kcm, (uint64_t)t * F + f);
            double v1 = ((double)(q >> 32) + 1.0) / 4294967296.0;
            double v2 = (double)(uint32_t)q / 4294967296.0;
            double rr = sqrt(-2.0 * log(v1));
            xr += ev->amplitude * rr * cos(2.0 * M_PI * v2);
            xi += ev->amplitude * rr * sin(2.0 * M_PI * v2);
          } else if (ev->kind == SYN_NOISE) {
            uint64_t q = syn_draw(knoise, base + i);
            double v1 = ((double)(q >> 32) + 1.0) / 4294967296.0;
            double v2 = (double)(uint32_t)q / 4294967296.0;
            double rr = sqrt(-2.0 * log(v1));
            xr += ev->amplitude * rr * cos(2.0 * M_PI * v2);
            xi += ev->amplitude * rr * sin(2.0 * M_PI * v2);
          }
        }
        row[i] = syn_encode(syn_clip_round(xr, C), syn_clip_round(xi, C));
      }
    }
  }
  return NULL;
}

/* Fill out[T][F][N]. Returns 0 on success. */
int synth_fill(const syn_desc* d, uint8_t* out, int nthreads) {
  const int N = d->n_inputs, NT = 2 * d->clip;
  if (N <= 0 || d->n_channels <= 0 || d->n_samples < 0 || d->clip < 1 || d->clip > 7) return -1;
  uint32_t* thr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N * NT);
  if (!thr) return -2;
  uint8_t* bin = (uint8_t*)malloc((size_t)N * 256);
  if (!bin) { free(thr); return -2; }
  for (int i = 0; i < N; ++i) {
    const uint32_t* th = thr + (size_t)i * NT;
    synth_thresholds(d->sigma[i], d->clip, thr + (size_t)i * NT);
    for (int hb = 0; hb < 256; ++hb) {
      uint32_t lo = (uint32_t)hb << 24, hi = lo | 0xFFFFFFu;
      int vlo = 0, vhi = 0;
      for (int k = 0; k < NT; ++k) { vlo += (th[k] <= lo); vhi += (th[k] <= hi); }
      bin[(size_t)i * 256 + hb] = (uint8_t)(vlo == vhi ? vlo : 0x80);
    }
  }
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  syn_job jobs[256];
  int64_t T = d->n_samples;
  for (int k = 0; k < nthreads; ++k) {
    jobs[k].d = d; jobs[k].out = out; jobs[k].thr = thr; jobs[k].bin = bin;
    jobs[k].t_begin = T * k / nthreads; jobs[k].t_end = T * (k + 1) / nthreads;
  }
  for (int k = 1; k < nthreads; ++k) pthread_create(&th[k], NULL, syn_worker, &jobs[k]);
  syn_worker(&jobs[0]);
  for (int k = 1; k < nthreads; ++k) pthread_join(th[k], NULL);
  free(thr);
  free(bin);
  /* Impulsive bursts: overwrite with round(A e^{i phi}) on every input. */
  const uint64_t kph = syn_key(d->seed, 3);
  for (int e = 0; e < d->n_events; ++e) {
    const syn_event* ev = &d->events[e];
    if (ev->kind != SYN_BURST) continue;
    for (int64_t t = ev->t0; t < ev->t1 && t < T; ++t)
      for (int i = 0; i < N; ++i) {
        double ph = 2.0 * M_PI * ((double)(syn_draw(kph, ((uint64_t)e << 40) + (uint64_t)t * N + i) >> 11) / 9007199254740992.0);
        out[((size_t)t * d->n_channels + ev->channel) * N + i] =
            syn_encode(syn_clip_round(ev->amplitude * cos(ph), d->clip), syn_clip_round(ev->amplitude * sin(ph), d->clip));
      }
  }
  return 0;
}
