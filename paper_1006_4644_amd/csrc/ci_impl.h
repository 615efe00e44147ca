// ci_impl.h -- internal structures shared by the host library and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ci.h"

namespace ci {

// Device-resident description of one data chunk.
struct SegDev {
  int64_t n;        // samples
  int64_t half;     // n / 2
  double fs, f_low, df;
  int32_t k_low;    // first band bin
  int32_t log2n;
  double g;         // power-of-two data scale folded into w
  double p_total;   // running sum at n/2 - 1
};

// Four-step factorisation n = N1 x N2 and the workgroup tiling.
struct Plan {
  int log2n;
  int n1, n2;       // pass 1: column DFTs of length n2 over k2 (one per k1)
                    // pass 2: column DFTs of length n1 over k1 (one per j2)
  int c;            // k1 columns per pass-1 workgroup
  int j;            // j2 columns per pass-2 workgroup
};

// The factorisation n = n1 n2 of a length for a precision: square, or
// n1 = 2 n2; at 2^21 the FP32 path takes n1 = n2 / 2 instead, so that its
// second pass can hand each 1024-point column to one wave.
Plan plan_for(int log2n, int c, int j, int precision);

// Slot sets of the intermediate and of the trigger bookkeeping in flight:
// batch b uses slot b % kSlots, so a batch's first pass can start while the
// finalisers of the previous kSlots - 1 batches still read their slots.
constexpr int kSlots = 3;

// Per-call trigger bookkeeping (device), kSlots slot sets.
struct TrigWork {
  unsigned long long* ppart;   // [kSlots][B][n2]    peak keys of the second pass
                               //                    (per workgroup or per wave)
  unsigned long long* wkeys;   // [kSlots][B][nwin]  window key per template
  unsigned long long* mkey;    // [kSlots][nwin]     merge key per window
  int* cnt;                    // [kSlots][B]        triggers per template
  int* sidx;                   // [kSlots][B][nwin]  staging slot of window w
  ci_trigger* stage;           // [kSlots][B][nwin]  compacted triggers
  ci_trigger* mrec;            // [nwin]             merged record per window
  unsigned long long* run;     // [1]                triggers placed so far
};

// Launch configuration of one search: tiles, pass-2 residency and batch.
struct Tune {
  int c = 8;             // k1 columns per pass-1 workgroup (4 or 8)
  int j = 4;             // j2 columns per pass-2 workgroup (4 or 8)
  int p2_per_cu = 2;     // resident pass-2 workgroups per CU (0: as many as fit)
  int64_t batch = 0;     // templates per batch (0: by intermediate size)
  int streams = 2;       // compute streams the batches alternate over (1 or 2)
  int p2_wave = 0;       // FP32 second pass with wave-owned columns (n1 512, 1024)
  bool tuned = false;    // chosen by the autotuner
};

// One instrumented launch: events bracketing it on its stream.
struct TimedLaunch {
  int kind;            // 0 pass 1, 1 pass 2
  int64_t templates;
  hipEvent_t e0, e1;
};

struct Seg;

// Host-side state.
struct Ctx {
  int device = 0;
  std::string err;
  int64_t batch_override = 0;
  // intermediate workspace (kSlots slot sets)
  void* ybuf = nullptr;
  size_t ybytes = 0;
  // trigger workspace
  void* tbuf = nullptr;
  size_t tbytes = 0;
  // two-polarization templates: per slot set the template transform
  // [B][n] complex64, then the sigma^2 partials [B][kTdChunks][2] doubles
  void* tdbuf = nullptr;
  size_t tdbytes = 0;
  // per-window records of ci_merge_triggers
  void* mbuf = nullptr;
  size_t mbytes = 0;
  size_t td_slot = 0;          // bytes per slot set of the current call
  // pinned staging for parameter upload
  void* pin = nullptr;
  size_t pinbytes = 0;
  hipEvent_t pin_ev = nullptr;
  bool pin_ev_armed = false;
  // internal streams: ws[0], ws[1] alternate the batches' two passes, ws[2]
  // runs the finalisers in batch order; events fork from and join back to
  // the caller's stream and order the slots
  hipStream_t ws[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[3] = {nullptr, nullptr, nullptr};
  hipEvent_t p2_done[kSlots] = {};   // second pass of the slot's batch done
  hipEvent_t fin_done[kSlots] = {};  // finaliser of the slot's batch done
  // launch configuration per (log2 n, precision): autotuned or default
  Tune tune[32][3];
  // live segments created on this context (detached when it is destroyed)
  std::vector<Seg*> segs;
  // live streams created on this context (released and detached when it
  // is destroyed)
  std::vector<struct ci_stream*> streams;
  // Ordering of the shared workspaces between calls: every call that uses
  // them waits for ws_free on its stream first and records it after its
  // last use, so calls on different streams (a ci_stream's internal
  // stream, a caller's streams) never overlap in the workspaces.
  hipEvent_t ws_free = nullptr;
  bool ws_free_armed = false;
  // bumped whenever a workspace is reallocated (cached graphs hold its
  // addresses)
  uint64_t ws_gen = 0;
  // graph replay of a schedule (ci_search_classes with CI_RUN_GRAPH): the
  // executable graph of the last captured schedule and the key of the
  // arguments it was captured with; captures run on cap_st
  hipStream_t cap_st = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<unsigned char> gkey;
  bool capturing = false;           // our own capture is in progress
  int64_t graph_captures = 0, graph_launches = 0;
  // device address of the no-allocation search's scratch on this device,
  // and whether such a call is being enqueued (no timing events then)
  void* scratch = nullptr;
  bool noalloc_call = false;
  // instrumentation
  bool timing = false;
  std::vector<TimedLaunch> launches;
  std::vector<hipEvent_t> ev_pool;
};

struct Seg {
  Ctx* ctx;          // owning context; null once that context is destroyed
  int device;        // HIP device of the segment's buffers
  ci_segment_spec spec;
  SegDev host;       // host copy (g and p_total are only valid on device)
  SegDev* dev;       // device copy
  float2* w;         // [n/2]  PSD-weighted, scaled data spectrum
  float2* w0;        // [n/2]  g x~ / S (two-polarization templates)
  double* isp;       // [n/2]  1 / S on the band, 0 below it
  double2* fpw;      // [n/2]  ((k df)^-7/3, (k df)^-7/6) on the band, 0 below
                     // it: fixed by n, fs and f_low, computed at creation
  double* psum;      // [n/2]  running sum of 4 df f^-7/3 / S from k_low
  double* bsum;      // [n/2 / kSegBlock] block sums, then block offsets
  float2* tw2048;    // [2048] exp(2 pi i e / 2048)
  double2* tw64;     // [2048] exp(2 pi i e / 2048) in FP64
  float2* twa;       // [2048] exp(2 pi i e / n)
  float2* twb;       // [n/2048] exp(2 pi i 2048 e / n)
  Plan plan;         // factorisation (tiles of the default configuration)
  uint4* mxa2[2];    // matrix-core fragments of the pass-2 column DFT (BF16, FP16):
                     // (n1/256 + 1) x 64 lanes x 4 x 16 bytes each
};

// Elements per workgroup of the segment-setup scan.
constexpr int kSegBlock = 2048;

// Kernel launchers (kernels.hip).
hipError_t launch_segment(Seg* s, const void* d_xtilde, const double* d_psd,
                          hipStream_t st);
// The segment's data-independent powers (fpw), once at creation.
hipError_t launch_segment_powers(Seg* s, hipStream_t st);
hipError_t launch_params(const Seg* s, ci_tparams* d_params, int64_t n,
                         void* d_htilde, hipStream_t st);
hipError_t launch_init_call(const TrigWork& tw, int nwin, int64_t* d_count,
                            hipStream_t st);
// Chi-squared veto of ntrig triggers (bands 2..64).
hipError_t launch_chisq(const Seg* s, const ci_tparams* d_params, int64_t ntmpl,
                        const ci_trigger* d_trig, int64_t ntrig, int bands, double* d_out,
                        hipStream_t st);
// Merge of two per-window trigger lists (at most one entry per window, the
// first min(count, cap) entries of each read) into `out` in window order:
// per window the larger rho^2, a's entry on equal values; b's template ids
// shifted by off_b; dense is nwin records of scratch.
hipError_t launch_merge(const ci_trigger* a, const int64_t* ca, int64_t cap_a, const ci_trigger* b,
                        const int64_t* cb, int64_t cap_b, int64_t off_b, int64_t nwin,
                        ci_trigger* dense, ci_trigger* out, int64_t cap, int64_t* d_count,
                        hipStream_t st);
// Streaming probe over `bytes` of buf: kind 0 writes, 1 reads, 2 copies the
// first half onto the second (bytes per half).
hipError_t launch_probe(int kind, void* buf, int64_t bytes, int blocks, hipStream_t st);
// Matrix-core operand tables of a segment (after its FP64 twiddles exist).
hipError_t launch_mx_tables(Seg* s, hipStream_t st);

struct BatchArgs {
  const Seg* seg;
  Plan plan;                  // factorisation and tiles of this call
  const ci_tparams* params;   // first template of the batch
  int64_t t0;                 // bank index of the first template
  int nb;                     // templates in this batch
  int slot;                   // slot set 0/1
  int bmax;                   // slot stride (templates per slot set)
  float2* y;                  // intermediate of this slot set
  // trigger mode
  TrigWork tw;
  int nwin;
  int64_t window;
  int64_t j_lo, j_hi;
  float thr2;
  ci_trigger* d_peaks;
  ci_trigger* d_trig;
  int64_t cap;
  int64_t* d_count;
  int merge;
  int last_batch;
  // series mode
  float2* d_z;                // first template's series
  int p2_per_cu;              // pass-2 workgroups per CU (0: as many as fit)
  int p2_wave;                // FP32 second pass with wave-owned columns
  int precision;              // CI_FP32 | CI_SPLIT_BF16 | CI_SPLIT_FP16
  // two-polarization templates (null td: the frequency-domain chirp)
  const ci_tdparams* td;      // batch's first template
  float2* uv;                 // [bmax][n] template transform of this slot set
  double* sig;                // [bmax][kTdChunks][2] sigma^2 partials
  // timing: when set, the next transform-pass launch records these at its
  // start and end
  hipEvent_t ev0, ev1;
};

hipError_t launch_pass1(const BatchArgs& a, bool zero_trig, hipStream_t st);
// Two-polarization templates of a batch: V = IDFT(u) of u = h_+ + i h_x
// (generated inside the transform's first pass) into a.uv, and the sigma^2
// partials in a.sig.  launch_pass1 then reads V when a.td is set.
hipError_t launch_td_prep(const BatchArgs& a, hipStream_t st);
// The generation step alone (u into a.uv).
hipError_t launch_td_gen(const BatchArgs& a, hipStream_t st);
// Spectra H~+ / H~x and sigma^2 of a prepared batch (either may be null).
hipError_t launch_td_export(const BatchArgs& a, void* d_hf, double* d_sigma2, hipStream_t st);
// Stream segment starting at global sample `start` of the device ring
// (capacity rmask + 1): spectrum xt [n/2 + 1], periodogram pg and PSD
// estimate psd [n/2 + 1] (half-width h); uv and y are [2][n] scratch.
hipError_t launch_stream_spectra(const Seg* seg, const float* ring, int64_t rmask, int64_t start,
                                 float2* uv, float2* y, float2* xt, double* pg, double* psd,
                                 int h, hipStream_t st);
// Mean PSD over the last cnt segments (ring of K estimates of m bins; the
// current one, in psd, goes to slot cur).
hipError_t launch_stream_avg(double* ring, int K, int cur, int cnt, int64_t m, double* psd,
                             hipStream_t st);
// sigma^2 partial sums per two-polarization template
constexpr int kTdChunks = 16;
hipError_t launch_pass2_trig(const BatchArgs& a, hipStream_t st);
hipError_t launch_pass2_series(const BatchArgs& a, hipStream_t st);
hipError_t launch_fin(const BatchArgs& a, hipStream_t st);
// hipSuccess when every kernel of a search with this plan and precision
// fits the per-workgroup LDS limit, hipErrorInvalidConfiguration when not.
hipError_t plan_fits(const Plan& p, int precision);
// Error of a call that has no context (read by ci_last_error(NULL)).
int report_error(int code, const char* msg);

}  // namespace ci
