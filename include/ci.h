/*
 * ci.h -- C ABI of the MI355X (gfx950) batched matched-filter library.
 *
 * The library runs the per-template search loop of Bosi, "cuInspiral"
 * (arXiv:1006.4644), section "Matched filtering": for every template of a
 * bank, generate the chirp, correlate it with one data chunk through the
 * coloured-noise inner product of eq. (matchedfilter), combine both
 * quadratures, keep the maxima above a threshold, and reduce the candidates
 * of all templates to local maxima.  The function split follows the
 * section "Pipeline main details":
 *
 *   ci_make_bank        bank file + host_template_init     (host only)
 *   ci_gen_templates    device_template_init + device_template_proc
 *   ci_matched_filter   device_complex_mf + device_cufft_C2R + device_madd2
 *   ci_find_triggers    device_maxfind + the clusterization step
 *   ci_chisq            the chi-squared veto planned in the Conclusions
 *   ci_td_*             the paper's own template form: time-domain
 *                       generator, two polarizations, two C2R + madd2
 *   ci_stream_*         the per-chunk loop over a continuous stream
 *   ci_bank_metric,     template placement at a set mismatch
 *   ci_make_bank_lattice
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns an int32 status (CI_OK or a negative CI_E* code).
 *   Argument and shape errors are detected synchronously and leave a
 *   message readable through ci_last_error().  HIP launch failures map to
 *   CI_EHIP.
 * - GPU work is enqueued asynchronously on the caller's hipStream_t (passed
 *   as void*; NULL means the default stream).  The library does not
 *   synchronise the caller's stream; results are valid after the caller
 *   synchronises.  Calls that block instead: ci_autotune, the *_destroy
 *   calls, the ci_stream_* calls as each documents, and any call whose
 *   context workspace has to grow (it waits for the device before
 *   releasing the old buffer; workspaces only grow, so this happens on the
 *   first calls at a new size).
 * - The caller owns every buffer it passes.  No call keeps a caller pointer
 *   after it returns.  The library owns only ci_ctx and ci_segment objects
 *   and their device workspaces, released by the matching *_destroy call.
 * - "d_" arguments are device pointers (hipMalloc'd or torch CUDA tensors);
 *   "host" arguments are host pointers.
 * - One ci_ctx per host thread.  The context's workspaces (intermediate,
 *   trigger bookkeeping) are shared by its calls: every call that uses
 *   them is ordered on the device after the previous such call (an event
 *   the library records on each call's stream), whatever streams they run
 *   on, including a ci_stream's internal stream.  Calls that a caller
 *   captures into its own graph skip that ordering (the graph's order
 *   applies), and a workspace cannot grow inside such a capture (CI_EINVAL;
 *   make the same call once outside the capture first).
 *   A segment passed with a ctx must have been created on that ctx
 *   (CI_EINVAL otherwise).
 * - Frequencies f_k = k fs/n, k = 0..n/2; df = fs/n; T = n/fs.
 * - Spectra are one-sided.  The inner product is
 *   <a, b> = 4 Re sum_k df a_k conj(b_k) / S_k (eq. (matchedfilter) taken at
 *   positive frequencies), summed over the template band
 *   k_low = ceil(f_low T) <= k <= k_high = min(floor(f_isco T), n/2 - 1),
 *   f_isco = 1 / (6^{3/2} pi M).
 */
#ifndef CI_H
#define CI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CI_OK 0
#define CI_EINVAL (-1)        /* bad argument or shape                     */
#define CI_ENOMEM (-2)        /* device or host allocation failed          */
#define CI_EHIP (-3)          /* a HIP runtime call or launch failed       */
#define CI_ETRUNC (-4)        /* capacity overflow seen on the host       */
#define CI_EUNSUPPORTED (-5)  /* valid request the library does not handle */

/* arithmetic of the inverse transform */
#define CI_FP32 0        /* FP32 VALU butterflies, FP32 intermediate        */
#define CI_SPLIT_BF16 1  /* the radix-16 stages of the second transform
                            pass as DFT-matrix products on MFMA, hi/lo BF16
                            operands, 3 products, FP32 accumulate; the first
                            pass in FP32 on the vector units; intermediate
                            stored as FP16 pairs (4 bytes per complex value:
                            half the transform's HBM bytes).  SNR error
                            below 1e-3 of the series maximum.             */
#define CI_SPLIT_FP16 2  /* the same with hi/lo FP16 operands (inputs scaled
                            by 2^6; |z| up to ~1e3 in SNR units)            */

/* bank kinds for ci_make_bank */
#define CI_BANK_GRID 0
#define CI_BANK_UNIFORM 1
#define CI_BANK_LOGUNIFORM 2

/* template flags (ci_tparams.flags) */
#define CI_TMPL_EMPTY 1  /* chirp ends below f_low: no band, no output     */

typedef struct ci_ctx ci_ctx;          /* opaque: device, workspaces, last error */
typedef struct ci_segment ci_segment;  /* opaque: one data chunk on one grid     */

/* One point of the template bank, in solar masses.  The mass-space grid of
 * the "Matched filtering" section: one (m1, m2)_i per template. */
typedef struct {
  double m1, m2;
} ci_template;

typedef struct {
  int32_t kind;      /* CI_BANK_GRID | CI_BANK_UNIFORM | CI_BANK_LOGUNIFORM */
  int32_t reserved;  /* must be 0 */
  double m_min, m_max;
  uint64_t seed;     /* ignored by CI_BANK_GRID */
} ci_bank_spec;

typedef struct {
  int64_t n;         /* samples per chunk: a power of two, 2^16 .. 2^21 */
  double fs;         /* sample rate, Hz */
  double f_low;      /* lower frequency cutoff, Hz (1 <= ceil(f_low T) < n/2) */
} ci_segment_spec;

/* One trigger: sample index, rho^2 = |z|^2/sigma^2 and the complex SNR
 * z/sigma at that sample (real part: the 0-phase quadrature correlator,
 * imaginary part: the pi/2 quadrature).  32 bytes. */
typedef struct {
  int64_t tmpl;      /* bank index, -1 if none */
  int64_t index;     /* sample index j in [0, n), -1 if none */
  float rho2;
  float re, im;
  int32_t window;    /* index / W, -1 if none */
} ci_trigger;

/* Per-template generator constants (the paper's host_template_init output),
 * device-resident, 96 bytes, plain old data.  Phase in revolutions:
 *   Psi_k / (2 pi) = -1/8 + c0 u^5 + c2 u^3 + c3 u^2 + c4 u,
 *   u = (x0 k)^{-1/3} = 1 / v_k,  v_k = (pi M f_k)^{1/3},
 * the restricted 2PN stationary-phase chirp with t_c = phi_c = 0. */
typedef struct ci_tparams {
  double m1, m2;          /* canonical masses, m1 >= m2 */
  double x0;              /* pi M df, M = (m1 + m2) G Msun / c^3 */
  double c0, c2, c3, c4;  /* phase coefficients, revolutions */
  double sigma2;          /* <h, h> of the unit-amplitude template */
  double tau;             /* 2PN chirp duration from f_low, seconds */
  float scale;            /* 4 df / (sigma g): g is the chunk's data scale */
  int32_t k_low, k_high;  /* band; k_high < k_low for an empty template */
  int32_t flags;          /* CI_TMPL_* */
  int32_t reserved[2];
} ci_tparams;

/* Constants of one two-polarization time-domain template (the paper's own
 * generator: phase of post-Newtonian order 2.5, Newtonian amplitude), made
 * by ci_td_params, device-resident, 176 bytes.  TaylorT2 from energy
 * balance with the published 2PN binding energy and 2.5PN flux, t_c = 0:
 *   t(v)   = -K v^-8 (1 + tau_2 v^2 + tau_3 v^3 + tau_4 v^4 + tau_5 v^5),
 *   dt/dv  = 8 K v^-9 (1 + r_2 v^2 + r_3 v^3 + r_4 v^4 + r_5 v^5),
 *   phi(v) = -P (v^-5 (1 + p_2 v^2 + p_3 v^3 + p_4 v^4) + p_5 ln v),
 * K = 5M/(256 eta), P = 1/(32 eta), phi the orbital phase.  Sample m >= 1
 * before coalescence (time -m/fs, index n - m of the circular grid) holds
 * h_+ + i h_x = v^2 exp(2 i phi(v)) with t(v) = -m/fs, for m_lo <= m <= m_hi
 * (v from v_low = (pi M f_low)^{1/3} to the ISCO v_end = 6^{-1/2}); the
 * statistic's band is k_low <= k <= n/2 - 1. */
typedef struct ci_tdparams {
  double m1, m2;          /* canonical masses, m1 >= m2 */
  double K;               /* 5 M / (256 eta), seconds */
  double tau[4];          /* tau_2 .. tau_5 */
  double r[4];            /* r_2 .. r_5 */
  double P;               /* 1 / (32 eta) */
  double p[4];            /* p_2 .. p_5 */
  double v_low, v_end;
  int64_t m_lo, m_hi;     /* chirp samples; m_hi < m_lo for an empty template */
  int32_t k_low, k_high;  /* band of the statistic */
  int32_t flags;          /* CI_TMPL_EMPTY */
  int32_t reserved;
} ci_tdparams;

/* --- context ------------------------------------------------------------ */

/* Create a context bound to HIP device `device`.  *out receives the handle.
 * Environment overrides, applied to the new context (a value that the
 * corresponding setter would reject fails the call with CI_EINVAL and no
 * context):
 *   CI_BATCH=<templates>   as ci_set_batch;
 *   CI_TUNE=<log2n>:<precision>:<tile_c>,<tile_j>,<p2_per_cu>,<batch>,
 *           <streams>[,<p2_wave>]   as ci_set_tune, entries separated by ';'
 *           (precision 0 FP32, 1 split BF16, 2 split FP16). */
int ci_ctx_create(int device, ci_ctx** out);
/* Frees the context's workspaces.  Segments created on it that are still
 * alive are detached: their buffers stay valid until ci_segment_destroy,
 * the only call that accepts them afterwards (others return CI_EINVAL). */
int ci_ctx_destroy(ci_ctx* ctx);

/* Message of the last failed call on `ctx` (or, with ctx == NULL, of the
 * last failed context-free call on this thread).  Valid until the next call. */
const char* ci_last_error(const ci_ctx* ctx);

/* Library version string. */
const char* ci_version(void);

/* --- bank (host only) ----------------------------------------------------
 * The template grid of the "Matched filtering" section.  GRID: g = ceil(
 * sqrt(n)) masses evenly spaced on [m_min, m_max], template t takes
 * (m[t / g], m[t % g]).  UNIFORM / LOGUNIFORM: m1 and m2 of template t are
 * draws 2t and 2t+1 of the counter-based SplitMix64 generator (Steele, Lea
 * & Flood 2014): u = (mix(seed + (i+1) 0x9E3779B97F4A7C15) >> 11) 2^-53,
 * m = m_min + u (m_max - m_min) or m = m_min exp(u log(m_max / m_min)).
 * Pairs are canonicalised to m1 >= m2.  Writes n entries to out_host.
 * CI_EINVAL when 0 < m_min <= m_max fails or n < 0. */
int ci_make_bank(const ci_bank_spec* spec, int64_t n, ci_template* out_host);

/* --- segment --------------------------------------------------------------
 * Prepare one data chunk (the "input data chunk" that device_complex_mf
 * correlates with).  d_xtilde: complex64[n/2+1] (interleaved re, im), the
 * data spectrum x~_k = dt sum_j x_j exp(-2 pi i jk/n).  d_psd: float64
 * [n/2+1], the one-sided noise PSD S_k > 0 on [k_low, n/2-1] (other bins
 * are ignored).  Both are read on `stream` before the call's work
 * completes and are not retained.  The segment holds the PSD-weighted
 * spectrum g x~_k f_k^{-7/6} / S_k (complex64; g a power of two) and the
 * FP64 running sum of 4 df f_k^{-7/3} / S_k from k_low, from which every
 * template's sigma^2 is one lookup.
 * CI_EINVAL for a non-power-of-two n, n outside 2^16..2^21, or a band
 * that is empty. */
int ci_segment_create(ci_ctx* ctx, const ci_segment_spec* spec,
                      const void* d_xtilde, const double* d_psd, void* stream,
                      ci_segment** out);
int ci_segment_destroy(ci_segment* seg);

/* Recompute a segment in place from a new data chunk and PSD on the same
 * grid (same n, fs, f_low): no allocation, asynchronous on `stream`.
 * Templates generated on the segment must be regenerated (sigma^2 depends
 * on the PSD). */
int ci_segment_update(ci_segment* seg, const void* d_xtilde, const double* d_psd,
                      void* stream);

/* --- templates -------------------------------------------------------------
 * Generator constants for n bank entries on `seg`'s grid (the paper's
 * host_template_init + device_template_init), and optionally the templates
 * themselves (device_template_proc).  bank_host: n ci_template (host),
 * copied before return.  d_params: ci_tparams[n] (device), written on
 * `stream`; sigma2 and scale are computed on the device from the segment's
 * FP64 running sum.  d_htilde_opt: NULL, or complex64[n][n_seg/2+1] that
 * receives h~_k = f_k^{-7/6} exp(-i Psi_k) inside the band and 0 outside
 * (unit amplitude, t_c = phi_c = 0).  The search itself never materialises
 * templates.  CI_EINVAL for non-positive masses. */
int ci_gen_templates(ci_ctx* ctx, const ci_segment* seg,
                     const ci_template* bank_host, int64_t n,
                     ci_tparams* d_params, void* d_htilde_opt, void* stream);

/* --- matched filter: the complex SNR series ---------------------------------
 * For each of n templates, z_j / sigma for j = 0..n_seg-1, where
 *   z_j = sum_{k=k_low}^{k_high} 4 df x~_k conj(h~_k) / S_k exp(2 pi i jk/n),
 * i.e. both quadrature correlators at every lag (eq. (matchedfilter)) in
 * SNR units: |z_j|^2 / sigma^2 is the quadrature sum c_+^2 + c_x^2.
 * d_z: complex64[n][n_seg] (device).  precision: CI_FP32, CI_SPLIT_BF16 or
 * CI_SPLIT_FP16 (the matrix-core stages).  An empty template yields zeros. */
int ci_matched_filter(ci_ctx* ctx, const ci_segment* seg,
                      const ci_tparams* d_params, int64_t n, int32_t precision,
                      void* d_z, void* stream);

/* --- search: peaks and threshold triggers ------------------------------------
 * The hot path.  Runs the same filter as ci_matched_filter without storing
 * the series and, per template t, reports:
 *  - d_peaks[t]: the largest rho^2 over samples j in [j_lo, j_hi) (ties to
 *    the smallest j), with z/sigma at that sample; index -1 for an empty
 *    template.
 *  - threshold triggers: for every aligned window [wW, (w+1)W) intersected
 *    with [j_lo, j_hi), the window's argmax m_w (ties to the smallest index)
 *    when rho2[m_w] > snr_threshold^2 (strict, the paper's c(t) > lambda).
 * merge_across_templates == 0: d_trig receives every (template, window)
 *   trigger, ordered by (template, window).
 * merge_across_templates != 0: d_trig receives one entry per window that has
 *   any trigger, the one with the largest rho^2 over all templates (ties to
 *   the smaller template id), ordered by window (the reduction of the
 *   candidate set to local maxima).
 * d_count (int64, device): receives the total number of triggers.  When it
 * exceeds `cap`, only the first `cap` in the stated order are written; the
 * call still returns CI_OK (the count exists only on the device once the
 * stream has run: compare *d_count with cap after synchronising).
 * rho2 of a trigger is the value that decided it; re/im are recomputed at
 * that index from the same transform's intermediate with FP64 accumulation.
 * window: W >= 1.  j_hi <= 0 means n_seg.  precision as for
 * ci_matched_filter. */
int ci_find_triggers(ci_ctx* ctx, const ci_segment* seg,
                     const ci_tparams* d_params, int64_t n, int32_t precision,
                     float snr_threshold, int64_t window, int64_t j_lo,
                     int64_t j_hi, ci_trigger* d_peaks, ci_trigger* d_trig,
                     int64_t cap, int64_t* d_count,
                     int32_t merge_across_templates, void* stream);

/* --- merge of per-window trigger lists ---------------------------------------
 * The reduction of the candidates to local maxima ("Matched filtering", the
 * final step of the per-chunk pipeline) across calls that each searched
 * part of one bank on the same segment (chunks of a large bank): d_a and
 * d_b are merged lists as ci_find_triggers with merge_across_templates
 * writes them (at most one entry per window, in window order); only their
 * first min(*count, cap) entries are read.  d_out receives, per window
 * w < nwin present in either, the entry with the larger rho2; on equal
 * rho2 the one from d_a (call it with the earlier chunk as d_a to keep
 * ties on the smaller template, as one call over the whole bank does).
 * d_b's template ids are shifted by tmpl_offset_b (the bank index of its
 * first template); d_a's are kept.  Window order; *d_count receives the
 * number of windows, and only the first cap entries are written.  d_out
 * may be d_a (accumulate in place) and d_count may be d_count_a.
 * Asynchronous on `stream`; uses the context's workspace (nwin records). */
int ci_merge_triggers(ci_ctx* ctx, const ci_trigger* d_a, const int64_t* d_count_a,
                      int64_t cap_a, const ci_trigger* d_b, const int64_t* d_count_b,
                      int64_t cap_b, int64_t tmpl_offset_b, int64_t nwin, ci_trigger* d_out,
                      int64_t cap, int64_t* d_count, void* stream);

/* --- search without allocation -----------------------------------------------
 * For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same search as ci_find_triggers, same arguments, same results bit for
 * bit, with every intermediate in a fixed device scratch area of 64 MiB per
 * GPU (a file-scope device array of the library, held until the process
 * ends) instead of the context's workspaces.  The call allocates nothing and
 * creates no stream or event: all launches go on `stream`, in order, in
 * batches of as many templates as fit the scratch (2 at n_seg = 2^20,
 * 1 at 2^21), so it is slower than ci_find_triggers.  CI_EINVAL when even
 * one template per batch does not fit (n_seg times 24 bytes plus the
 * trigger bookkeeping of n_seg / window windows).  Every such call on one
 * GPU shares that GPU's scratch: calls that overlap on the device (other
 * streams, other contexts, other host threads) race and give wrong
 * results; order them.  Timing (ci_set_timing) does not record these
 * launches. */
int ci_find_triggers_noalloc(ci_ctx* ctx, const ci_segment* seg,
                             const ci_tparams* d_params, int64_t n, int32_t precision,
                             float snr_threshold, int64_t window, int64_t j_lo,
                             int64_t j_hi, ci_trigger* d_peaks, ci_trigger* d_trig,
                             int64_t cap, int64_t* d_count,
                             int32_t merge_across_templates, void* stream);

/* --- the paper's two-polarization form ----------------------------------------
 * The template form of "Template generation" and of the per-template loop
 * of "Matched filtering": both polarizations generated in the time domain,
 * Fourier transformed, each normalised to unit norm (sigma_+^2 = <h_+, h_+>,
 * sigma_x^2 = <h_x, h_x>), correlated with the data through
 * eq. (matchedfilter), taken back to the time domain by two real inverse
 * transforms (the paper's two device_cufft_C2R) and combined in quadrature
 * (device_madd2):
 *   c_+(t_j) = 4 Re sum_{k_low <= k <= n/2-1} df x~_k conj(H~+_k) e^{2 pi i jk/n}
 *              / S_k / sigma_+,   likewise c_x,   rho^2 = c_+^2 + c_x^2,
 * with H~_k = dt sum_j h_j e^{-2 pi i jk/n}.  On the device the two real
 * transforms are one complex transform of the Hermitian-packed spectrum
 * (its real part is c_+, its imaginary part c_x), and the two forward
 * transforms are one complex transform of u = h_+ + i h_x.  FP32 arithmetic
 * (FP64 for v(t), the phase and sigma^2); no split-precision variant.
 *
 * ci_td_params (bank on the host, outputs on the device): d_tdparams[n],
 * asynchronous on `stream`; CI_EINVAL for a non-positive mass. */
int ci_td_params(ci_ctx* ctx, const ci_segment* seg, const ci_template* bank_host,
                 int64_t n, ci_tdparams* d_tdparams, void* stream);

/* Materialise templates (tests, inspection).  Any output may be NULL:
 *   d_u      complex64 [n][n_seg]: h_+ + i h_x on the circular grid;
 *   d_hf     complex64 [n][2][n_seg/2 + 1]: H~+_k then H~x_k, k = 0..n_seg/2;
 *   d_sigma2 double [n][2]: sigma_+^2, sigma_x^2 (0 for an empty template).
 * Uses the context's workspace. */
int ci_td_templates(ci_ctx* ctx, const ci_segment* seg, const ci_tdparams* d_tdparams,
                    int64_t n, void* d_u, void* d_hf, double* d_sigma2, void* stream);

/* Series: d_z complex64 [n][n_seg] receives c_+ + i c_x (zero for an empty
 * template). */
int ci_td_matched_filter(ci_ctx* ctx, const ci_segment* seg, const ci_tdparams* d_tdparams,
                         int64_t n, void* d_z, void* stream);

/* Search with the two-polarization statistic: arguments, outputs, ordering,
 * merge and error behaviour as ci_find_triggers (FP32); re/im of a trigger
 * are c_+ and c_x at its sample. */
int ci_td_find_triggers(ci_ctx* ctx, const ci_segment* seg, const ci_tdparams* d_tdparams,
                        int64_t n, float snr_threshold, int64_t window, int64_t j_lo,
                        int64_t j_hi, ci_trigger* d_peaks, ci_trigger* d_trig, int64_t cap,
                        int64_t* d_count, int32_t merge_across_templates, void* stream);

/* --- continuous stream processing ---------------------------------------------
 * The per-chunk loop of "Matched filtering" run over a continuous strain
 * stream: overlap-save segments of n samples with stride n/2 (segment s
 * covers global samples [s n/2, s n/2 + n)), each searched over its valid
 * half j in [n/4, 3n/4), so that consecutive valid regions tile the stream
 * once and chirps up to n/4 samples long need no wrap-around.  Per segment,
 * on the device: the spectrum x~_k = dt sum_j x_j e^{-2 pi i jk/n}; the PSD
 * estimate, the Hann-windowed periodogram P_k = 2 |X_k|^2 / (T 3/8),
 * X_k = dt sum_j sin^2(pi j/n) x_j e^{-2 pi i jk/n}, averaged over the
 * in-band bins [k - h, k + h] intersected with [k_low, n/2 - 1] (S_k = 0
 * outside that band), optionally averaged with the estimates of the
 * previous segments (psd_segments); the segment update, the templates'
 * sigma^2 and the
 * merged search of ci_find_triggers (at the spec's precision, the
 * context's launch configuration).  Trigger indices and windows are global.
 * Host samples are staged through pinned memory and copied on a stream of
 * their own, so copies overlap the search of earlier segments. */
typedef struct ci_stream ci_stream;  /* opaque */

typedef struct {
  int64_t n;              /* segment length: power of two, 2^16 .. 2^21 */
  double fs, f_low;
  int32_t psd_half_width; /* h: 0 .. 256 */
  float snr_threshold;    /* lambda (rho^2 > lambda^2 triggers) */
  int64_t window;         /* W: 1 .. n/4, dividing n/4 (each window inside
                             one segment's valid region [n/4, 3n/4)) */
  int64_t cap;            /* merged triggers kept per segment, >= 1 */
  int32_t psd_segments;   /* K: the PSD used for a segment is the mean of
                             the estimates of it and the K - 1 before it
                             (fewer at the start); 0 or 1: its own; <= 16 */
  int32_t precision;      /* of the search: CI_FP32 | CI_SPLIT_BF16 |
                             CI_SPLIT_FP16 (the segment transform and the
                             PSD estimate are FP32 / FP64 either way) */
} ci_stream_spec;

/* bank_host[n_templates] is copied.  CI_EINVAL for a bad spec or bank. */
int ci_stream_create(ci_ctx* ctx, const ci_stream_spec* spec, const ci_template* bank_host,
                     int64_t n_templates, ci_stream** out);
/* Waits for the stream's work, frees it.  Destroy a stream before its
 * context. */
int ci_stream_destroy(ci_stream* s);
/* Append `count` samples (host, float32) and enqueue every segment they
 * complete.  Returns once the samples are staged; may wait for earlier
 * copies and, when two segments are already in flight, for the older. */
int ci_stream_push(ci_stream* s, const float* host_x, int64_t count);
/* Collect triggers of finished segments, in segment order (so in global
 * window order): host_out[0 .. *n_out) receives at most `cap`; the rest
 * stay queued for the next call.  wait != 0 first waits for every
 * enqueued segment.  *segments_done (may be NULL): segments collected so
 * far.  A segment whose merged list overflowed its cap contributes its
 * first `cap` windows and sets bit 0 of *flags (may be NULL). */
int ci_stream_poll(ci_stream* s, int32_t wait, ci_trigger* host_out, int64_t cap,
                   int64_t* n_out, int64_t* segments_done, int32_t* flags);
/* Inspection: waits for the stream's work and copies the spectrum
 * (complex64 [n/2 + 1]) and PSD estimate (double [n/2 + 1]) of the last
 * segment processed to device buffers (either may be NULL); *segment
 * receives its index (-1 before the first). */
int ci_stream_last(ci_stream* s, void* d_xtilde, double* d_psd, int64_t* segment);

/* --- template-bank placement ---------------------------------------------------
 * The bank of "Matched filtering" placed so that every point of the mass
 * range loses at most a set fraction of SNR to its nearest template (the
 * paper's footnote: 2-5 % mismatch).  Coordinates: the chirp times at
 * f_0 = f_low,
 *   tau_0 = 5 / (256 pi f0 eta) (pi M f0)^{-5/3},  tau_3 = 1 / (8 f0 eta) (pi M f0)^{-2/3}.
 * Metric (Owen, PRD 53, 6749 (1996)): with w(f) = f^{-7/3}/S on the
 * template's band of the grid (n, fs), J the w-weighted mean, psi_a the
 * derivative of the 2PN stationary phase along tau_a and C the
 * J-covariance of (2 pi f, psi_0, psi_3),
 *   gamma_ab = (1/2) (C_ab - C_at C_bt / C_tt),   1 - match ~ gamma_ab dtau^a dtau^b,
 * the match maximised over phase and (continuous) time.  Host only.
 *
 * ci_bank_metric: gamma_out = {g_00, g_03, g_33} at (m1, m2); psd_host
 * [n/2 + 1].  CI_EINVAL for bad masses or an empty band. */
int ci_bank_metric(const double* psd_host, int64_t n, double fs, double f_low, double m1,
                   double m2, double* gamma_out);

typedef struct {
  double m_min, m_max;   /* component masses, 0 < m_min < m_max */
  double min_match;      /* e.g. 0.97 for 3 % mismatch, in (0.5, 1) */
} ci_lattice_spec;

/* Hexagonal lattice in (tau_0, tau_3) for the mass range
 * m_min <= m2 <= m1 <= m_max.  The metric is sampled over the range; in
 * each of 12 strips of log tau_0 (fewer when the range is less than 120
 * covering radii long along tau_0) a constant metric G is taken, the one of
 * least determinant that bounds every sample of the strip (G - g positive
 * semi-definite), times 1.05; lattice points with covering radius
 * sqrt(1 - min_match) (side sqrt(3 (1 - min_match))) in G cover the strip,
 * those outside it but within the covering radius are moved to the
 * nearest point of its boundary.  out_host[0 .. min(count, cap)) receives
 * (m1, m2) with m1 >= m2; *count the number placed (CI_ETRUNC when above
 * cap; cap = 0 and out_host = NULL query the count).  The metric samples
 * and the lattice rows are computed on up to 16 host threads, joined in a
 * fixed order: the result does not depend on the thread count.  Safe to
 * call from several threads at once. */
int ci_make_bank_lattice(const ci_lattice_spec* spec, const double* psd_host, int64_t n,
                         double fs, double f_low, ci_template* out_host, int64_t cap,
                         int64_t* count);

/* --- chi-squared veto ---------------------------------------------------------
 * The signal-consistency test the Conclusions plan as the next stage of the
 * pipeline (their ref. [Chi2], B. Allen, Phys. Rev. D 71, 062001 (2005)),
 * evaluated at trigger samples.  For trigger i with template t = tmpl and
 * sample j = index:
 *  - the band [k_low, k_high] of t splits into p = `bands` contiguous bands
 *    of equal sigma^2 share: with c_k the running sum of 4 df f^{-7/3}/S
 *    over [k_low, k], edge e_l (0 < l < p) is the first k with
 *    c_k >= (l / p) c_{k_high}; e_0 = k_low, e_p = k_high + 1;
 *  - z_l is the series value z(j)/sigma of ci_matched_filter restricted to
 *    band l (so z = sum_l z_l), accumulated in FP64 from the segment's
 *    weighted spectrum and the chirp phase at each bin;
 *  - d_chisq[i] = p sum_l |z_l - z/p|^2, which in Gaussian noise follows a
 *    chi-squared law with 2p - 2 degrees of freedom and stays small for a
 *    signal that matches the template.
 * d_params: [n] generated on seg (device).  d_trig: [n_trig] device, e.g.
 * the d_trig or d_peaks output of ci_find_triggers; d_chisq: [n_trig]
 * doubles, device, owned by the caller.  A trigger whose tmpl is outside
 * [0, n) or whose index is outside [0, n_seg), and one of an empty
 * template, gets NaN.  bands: 2..64, else CI_EINVAL.  Asynchronous on
 * `stream`; no workspace. */
int ci_chisq(ci_ctx* ctx, const ci_segment* seg, const ci_tparams* d_params,
             int64_t n, const ci_trigger* d_trig, int64_t n_trig,
             int32_t bands, double* d_chisq, void* stream);

/* --- batch schedule: length classes -----------------------------------------
 * A bank of uneven chirp lengths is searched in length classes: each
 * template goes to the shortest segment whose duration n_c / fs covers its
 * 2PN time to coalescence from f_low (the paper's per-chunk loop over a
 * bank, with the chunk length matched to the template).
 * ci_length_classes (host only): class_n[0..nclass-1], increasing powers of
 * two; class_out[i] receives the index c of the smallest class_n[c] with
 * tau_2PN(f_low; m1, m2) <= class_n[c] / fs, or nclass - 1 when none is
 * long enough.  CI_EINVAL for non-positive masses or a bad class list. */
int ci_length_classes(const ci_template* bank_host, int64_t n, double fs,
                      double f_low, const int64_t* class_n, int32_t nclass,
                      int32_t* class_out);

/* One class of a multi-class search: the same arguments as one
 * ci_find_triggers call (all pointers device, owned by the caller). */
typedef struct {
  const ci_segment* seg;        /* data chunk of the class's length */
  const ci_tparams* d_params;   /* [n] generated on seg */
  int64_t n;
  int64_t j_lo, j_hi;           /* search range; j_hi <= 0 means n_seg */
  ci_trigger* d_peaks;          /* [n] */
  ci_trigger* d_trig;           /* [cap] */
  int64_t cap;
  int64_t* d_count;             /* [1] */
} ci_class_job;

/* Run every job of the schedule, with results identical to one
 * ci_find_triggers call per job (same precision, threshold, window and
 * merge flag; merging is within a job).  Batches of all jobs alternate
 * between the context's two internal compute streams (their finalisers
 * run in order on a third), so consecutive batches overlap across class
 * boundaries; `stream` waits for all of them.
 * Jobs share the context's workspace; the library orders calls on one
 * context against each other on the device (see ci_ctx_create).
 * flags: 0, or CI_RUN_GRAPH: the whole schedule runs as one HIP graph
 * launch on `stream`: a chain of kernel nodes (the calls' initialisation,
 * then per batch its first pass, second pass and finaliser, in order; the
 * eager schedule's overlap of consecutive batches on two streams is not
 * kept).  The graph is captured on the first call
 * with a given set of arguments (jobs, output pointers, threshold, window,
 * merge, precision, launch configuration) and replayed by later calls
 * with the same set; any change recaptures it, and then waits for the
 * previous graph's last replay before releasing it.  Results are
 * identical to the eager schedule's.  Launches inside the graph are not
 * timed (ci_set_timing).  CI_EINVAL when `stream` is itself being
 * captured, or when the context workspace would have to grow during the
 * capture (it is sized before). */
#define CI_RUN_GRAPH 1
int ci_search_classes(ci_ctx* ctx, const ci_class_job* jobs, int32_t njobs,
                      int32_t precision, float snr_threshold, int64_t window,
                      int32_t merge_across_templates, int32_t flags,
                      void* stream);

/* Graphs captured and graph launches made by ci_search_classes with
 * CI_RUN_GRAPH on this context so far (either pointer may be NULL). */
int ci_graph_stats(ci_ctx* ctx, int64_t* captures, int64_t* launches);

/* --- tuning -----------------------------------------------------------------
 * Templates per batch of the two-pass transform for every length (0 = the
 * per-length configuration below).  The intermediate workspace is
 * 2 x batch x n_seg x 8 bytes. */
int ci_set_batch(ci_ctx* ctx, int64_t templates_per_batch);

/* Launch configuration of the search at transform length 2^log2n and one
 * precision, held per context.  The transform's arithmetic does not depend
 * on it: every configuration gives bit-identical results. */
typedef struct {
  int32_t log2n;        /* 16..21 */
  int32_t precision;    /* CI_FP32 | CI_SPLIT_BF16 | CI_SPLIT_FP16 */
  int32_t tile_c;       /* first-pass columns per workgroup: 4 or 8 */
  int32_t tile_j;       /* second-pass columns per workgroup: 4 or 8 */
  int32_t p2_per_cu;    /* resident second-pass workgroups per CU, 0..8
                           (0: as many as fit) */
  int32_t tuned;        /* out: 1 when chosen by ci_autotune */
  int64_t batch;        /* templates per batch, 0..4096 (0: 2^26 / n_seg,
                           limited by the trigger workspace) */
  double ms;            /* out (ci_autotune): time of the chosen one, ms */
  int32_t candidates;   /* out (ci_autotune): configurations timed */
  int32_t rejected;     /* out (ci_autotune): configurations excluded
                           because their output differed */
  int32_t streams;      /* compute streams the batches' passes alternate
                           over: 2 (one batch's second pass overlaps the
                           next batch's first) or 1 (in order); 0 means 2 */
  int32_t p2_wave;      /* FP32 second pass at n1 = 512 or 1024 (2^17 ..
                           2^21): 1 hands each column to one wave after its
                           first stage (one cross-wave exchange, per-wave
                           post-pass), 0 keeps the columns spread over the
                           workgroup; ignored elsewhere */
} ci_tune;

int ci_get_tune(ci_ctx* ctx, int32_t log2n, int32_t precision, ci_tune* out);
/* Sets tile_c, tile_j, p2_per_cu, batch, streams and p2_wave for (log2n,
 * precision). */
int ci_set_tune(ci_ctx* ctx, const ci_tune* cfg);

/* Autotuner: times ci_find_triggers (no merge) on the given templates under
 * a coordinate search over tiles, the FP32 second-pass variant (p2_wave),
 * second-pass residency, batch size and the number of compute streams
 * (the last step jointly over batch size and second-pass tile width),
 * starting from the default configuration; a candidate whose peaks,
 * trigger count or trigger list differ in any bit from the default's is
 * excluded.  Stores the fastest as the context's configuration for the
 * segment's length and precision and reports it in *out (may be NULL).
 * Blocking: synchronises `stream`; allocates and frees its own output
 * buffers (n + min(n * windows, 2^20) triggers). */
int ci_autotune(ci_ctx* ctx, const ci_segment* seg, const ci_tparams* d_params,
                int64_t n, int32_t precision, float snr_threshold,
                int64_t window, ci_tune* out, void* stream);

/* --- instrumentation ---------------------------------------------------------
 * With timing enabled, every transform-pass launch is bracketed by HIP
 * events recorded on its launch stream.  ci_kernel_times() waits for the
 * recorded events, reports per pass the number of launches, the templates
 * they processed and their summed duration in milliseconds, and clears the
 * record.  kind: 0 = pass 1 (generate + first pass), 1 = pass 2 (second
 * pass + post-pass). */
typedef struct {
  int64_t launches;
  int64_t templates;
  double ms;
} ci_kernel_time;

int ci_set_timing(ci_ctx* ctx, int32_t enable);

/* Streaming bandwidth of the device, for comparing the search's kernels
 * with what plain memory traffic reaches: kind 0 writes `bytes` of d_buf
 * (16-byte non-temporal stores), 1 reads them (16-byte non-temporal loads),
 * 2 copies the first `bytes` of d_buf onto the next `bytes` (d_buf holds
 * 2 x bytes).  Grid-stride loops over 8 workgroups of 256 lanes per compute
 * unit.  *gbs: the best of `reps` timed launches (after one warm-up), in
 * 1e9 bytes/s moved (read plus written for a copy).  Blocking; the buffer's
 * contents are overwritten (kinds 0 and 2).  bytes: a multiple of 16,
 * >= 4096. */
int ci_hbm_probe(ci_ctx* ctx, int32_t kind, void* d_buf, int64_t bytes, int32_t reps,
                 double* gbs);
int ci_kernel_times(ci_ctx* ctx, ci_kernel_time* pass1, ci_kernel_time* pass2);

#ifdef __cplusplus
}
#endif

#endif /* CI_H */
