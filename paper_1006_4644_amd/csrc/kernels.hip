// kernels.hip -- gfx950 kernels of the batched matched-filter search.
//
// Per template (the per-template loop of the "Matched filtering" section):
//   pass 1: generate the chirp bins on chip, form the correlator integrand
//           Z_k = 4 df x~_k conj(h~_k) / (S_k sigma), and run the first
//           four-step pass (column DFTs over k2 for a tile of k1), writing
//           the twiddled intermediate once;
//   pass 2: read it once, run the second pass (column DFTs over k1 for a
//           tile of j2), and reduce |z|^2 to the peak and the window
//           maxima above threshold on the fly (or store the series).
// Template normalisation (sigma^2) is one lookup in the chunk's FP64
// running sum; the chirp phase is evaluated in FP64 and reduced mod 2 pi
// before FP32 trigonometry.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "ci_impl.h"
#include "fft_device.h"
#include "mfma_device.h"

namespace ci {

typedef unsigned long long u64;

// ---------------------------------------------------------------------------
// chirp phase
// ---------------------------------------------------------------------------

// Fractional part (revolutions, in [-1/2, 1/2]) of Psi_k / (2 pi) for the
// restricted 2PN stationary-phase chirp with t_c = phi_c = 0:
//   Psi/(2 pi) = -1/8 + c0 u^5 + c2 u^3 + c3 u^2 + c4 u,  u = (x0 k)^{-1/3}.
// u starts from an FP32 estimate and takes one FP64 Newton step
// (u <- u (4 - x u^3) / 3), enough for ~1e-13 relative error; the
// polynomial and the reduction mod 1 are FP64, so the phase error stays
// below 1e-7 rad even where |Psi| reaches 1e5 rad.
__device__ __forceinline__ float phase_frac(const ci_tparams& P, int k) {
  const double x = P.x0 * (double)k;
  const float y0 = __builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf((float)x));
  double u = (double)y0;
  u = u * (4.0 - x * (u * u * u)) * (1.0 / 3.0);
  const double in = fma(u * u, P.c0, P.c2);
  const double t3 = fma(u, in, P.c3);
  const double t4 = fma(u, t3, P.c4);
  const double r = fma(u, t4, -0.125);
  return (float)(r - rint(r));
}

// (cos Psi_k, sin Psi_k) through the hardware sine/cosine, whose input is
// in revolutions (|error| <= 1.3e-7 on [-1/2, 1/2]).
__device__ __forceinline__ float2 chirp_phasor(const ci_tparams& P, int k) {
  const float fr = phase_frac(P, k);
  return make_float2(__builtin_amdgcn_cosf(fr), __builtin_amdgcn_sinf(fr));
}

// ---------------------------------------------------------------------------
// segment setup (once per data chunk)
// ---------------------------------------------------------------------------

// Segment setup in three deterministic FP64 steps over blocks of kSegBlock
// bins: (1) the terms 4 df f_k^{-7/3} / S_k on [k_low, n/2) and their
// block sums, (2) the scan of the block sums, the total and the data scale
// g, (3) the running sum inside each block plus the weighted spectrum.
constexpr int kSegThreads = 1024;
constexpr int kSegPer = kSegBlock / kSegThreads;

__device__ __forceinline__ double seg_term(int64_t k, int64_t kl, double df, const double* psd,
                                           const double2* fpw) {
  return k >= kl ? 4.0 * df * fpw[k].x / psd[k] : 0.0;
}

// fpw[k] = ((k df)^-7/3, (k df)^-7/6) for k >= k_low, else 0: the powers of
// the template norm and of the template amplitude, which depend only on the
// segment's length, sample rate and cut-off (computed once per segment).
__global__ __launch_bounds__(256) void k_seg_powers(const SegDev* __restrict__ sd,
                                                    double2* __restrict__ fpw) {
  const int64_t kl = sd->k_low, half = sd->half;
  const double df = sd->df;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < half;
       k += (int64_t)gridDim.x * blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    if (k >= kl) {
      const double f = (double)k * df;
      v = make_double2(pow(f, -7.0 / 3.0), pow(f, -7.0 / 6.0));
    }
    fpw[k] = v;
  }
}

// Exclusive scan of one double per lane over a 256-lane workgroup.
__device__ double block_excl_scan_d(double v, double* sh, double* total) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __syncthreads();
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const double u = (tid >= off) ? sh[tid - off] : 0.0;
    __syncthreads();
    sh[tid] += u;
    __syncthreads();
  }
  const double incl = sh[tid];
  *total = sh[nt - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kSegThreads) void k_seg_terms(const SegDev* __restrict__ sd,
                                                           const double* __restrict__ psd,
                                                           const double2* __restrict__ fpw,
                                                           double* __restrict__ psum,
                                                           double* __restrict__ bsum) {
  __shared__ double sh[kSegThreads];
  const int64_t kl = sd->k_low;
  const double df = sd->df;
  const int64_t base = (int64_t)blockIdx.x * kSegBlock + threadIdx.x * kSegPer;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kSegPer; ++i) {
    const double v = seg_term(base + i, kl, df, psd, fpw);
    psum[base + i] = v;
    s += v;
  }
  double tot;
  (void)block_excl_scan_d(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_seg_scan(SegDev* sd, double* __restrict__ bsum,
                                                   int nblk) {
  __shared__ double sh[1024];
  const int tid = threadIdx.x;
  const double v = tid < nblk ? bsum[tid] : 0.0;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const double u = (tid >= off) ? sh[tid - off] : 0.0;
    __syncthreads();
    sh[tid] += u;
    __syncthreads();
  }
  if (tid < nblk) bsum[tid] = sh[tid] - v;
  if (tid == 1023) {
    const double tot = sh[1023];
    sd->p_total = tot;
    // E|x~ f^{-7/6} / S|^2 = (T/2) f^{-7/3} / S for data with PSD S: scale
    // the weighted spectrum to unit mean power by an exact power of two.
    const double T = (double)sd->n / sd->fs;
    const double len = (double)(sd->half - sd->k_low);
    const double mean = 0.5 * T * (tot / (4.0 * sd->df)) / len;
    sd->g = exp2(rint(-0.5 * log2(mean)));
  }
}

__global__ __launch_bounds__(kSegThreads) void k_seg_final(const SegDev* __restrict__ sd,
                                                           const float2* __restrict__ xt,
                                                           const double* __restrict__ psd,
                                                           double* __restrict__ psum,
                                                           const double* __restrict__ boff,
                                                           float2* __restrict__ w,
                                                           float2* __restrict__ w0,
                                                           double* __restrict__ isp,
                                                           const double2* __restrict__ fpw) {
  __shared__ double sh[kSegThreads];
  const int64_t kl = sd->k_low;
  const double g = sd->g;
  const int64_t base = (int64_t)blockIdx.x * kSegBlock + threadIdx.x * kSegPer;
  double v[kSegPer];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kSegPer; ++i) {
    v[i] = psum[base + i];
    s += v[i];
  }
  double tot;
  double run = boff[blockIdx.x] + block_excl_scan_d(s, sh, &tot);
#pragma unroll
  for (int i = 0; i < kSegPer; ++i) {
    const int64_t k = base + i;
    run += v[i];
    psum[k] = k >= kl ? run : 0.0;
    float2 o = make_float2(0.f, 0.f), o0 = o;
    double is = 0.0;
    if (k >= kl) {
      is = 1.0 / psd[k];
      const double fac0 = g * is;
      const double fac = fac0 * fpw[k].y;
      const float2 x = xt[k];
      o = make_float2((float)((double)x.x * fac), (float)((double)x.y * fac));
      o0 = make_float2((float)((double)x.x * fac0), (float)((double)x.y * fac0));
    }
    w[k] = o;
    w0[k] = o0;
    isp[k] = is;
  }
}

// sigma^2 and the per-template scale 4 df / (sigma g).
__global__ __launch_bounds__(256) void k_params(const SegDev* __restrict__ sd,
                                                const double* __restrict__ psum,
                                                ci_tparams* __restrict__ prm, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  ci_tparams P = prm[i];
  if (P.flags & CI_TMPL_EMPTY) {
    P.sigma2 = 0.0;
    P.scale = 0.f;
  } else {
    P.sigma2 = psum[P.k_high];
    P.scale = (float)(4.0 * sd->df / (sqrt(P.sigma2) * sd->g));
  }
  prm[i] = P;
}

// Materialised templates h~_k = f^{-7/6} exp(-i Psi_k) in the band, 0 out.
__global__ __launch_bounds__(256) void k_htilde(const SegDev* __restrict__ sd,
                                                const ci_tparams* __restrict__ prm,
                                                float2* __restrict__ h) {
  const int64_t t = blockIdx.y;
  const ci_tparams P = prm[t];
  const int64_t m = sd->half + 1;
  float2* ht = h + t * m;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x) {
    float2 o = make_float2(0.f, 0.f);
    if (k >= P.k_low && k <= P.k_high) {
      const float2 e = chirp_phasor(P, (int)k);
      const float amp = (float)pow((double)k * sd->df, -7.0 / 6.0);
      o = make_float2(amp * e.x, -amp * e.y);
    }
    ht[k] = o;
  }
}

// ---------------------------------------------------------------------------
// workgroup -> tile mapping
// ---------------------------------------------------------------------------

// Consecutive workgroup ids are dealt round-robin over the 8 XCDs; remap
// them so that each XCD walks a contiguous range of tiles (neighbouring
// k1 tiles share cache lines of the weighted spectrum).
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  if ((nblk & 7) != 0) return bid;
  return (bid & 7) * (nblk >> 3) + (bid >> 3);
}

// ---------------------------------------------------------------------------
// pass 1: generate + correlate + first four-step pass
// ---------------------------------------------------------------------------

// w = 1/v with t(v) = t (t < 0) for a time-domain template.  In w the
// chirp time is a polynomial, t = -K w^3 (w^5 + tau_2 w^3 + tau_3 w^2 +
// tau_4 w + tau_5), so Newton's method needs no division: the residual is
// evaluated in FP64 and divided by the derivative through its FP32
// reciprocal, which still converges to FP64 accuracy (once close, each
// step shrinks the error by ~1e-7 or better).  Started from the Newtonian
// guess w = (-t / K)^{1/8}, kept inside [1/v_end, 1/v_low], until the step
// falls below 1e-15 w.
__device__ __forceinline__ double td_solve_w(const ci_tdparams& T, double t) {
  const float q = (float)(-t / T.K);
  const double wlo = 1.0 / T.v_end, whi = 1.0 / T.v_low;
  double w = (double)__builtin_amdgcn_exp2f(0.125f * __builtin_amdgcn_logf(q));
  w = fmin(fmax(w, wlo), whi);
  for (int it = 0; it < 40; ++it) {
    const double w2 = w * w;
    const double p = fma(w, fma(w, fma(w, fma(w, w, T.tau[0]), T.tau[1]), T.tau[2]), T.tau[3]);
    const double g = fma(-T.K * w2 * w, p, -t);
    const double dp = fma(w, fma(w, fma(w, fma(8.0 * w, w, 6.0 * T.tau[0]), 5.0 * T.tau[1]),
                                 4.0 * T.tau[2]),
                          3.0 * T.tau[3]);
    const float rc = __builtin_amdgcn_rcpf((float)(-T.K * w2 * dp));
    double wn = fma(-g, (double)rc, w);
    wn = fmin(fmax(wn, wlo), whi);
    const bool done = fabs(wn - w) <= 1e-15 * w;
    w = wn;
    if (done) break;
  }
  return w;
}

// Gravitational-wave phase 2 phi in revolutions from w = 1/v, reduced to
// [-1/2, 1/2] in FP64: 2 phi = -(2 P) (w^5 + p_2 w^3 + p_3 w^2 + p_4 w -
// p_5 log w), the TaylorT2 phase v^-5 (1 + p_2 v^2 + p_3 v^3 + p_4 v^4) +
// p_5 log v written in w.
__device__ __forceinline__ float td_phase_frac(const ci_tdparams& T, double w) {
  const double poly = w * fma(w, fma(w, fma(w, w, T.p[0]), T.p[1]), T.p[2]);
  const double phi = -T.P * fma(-T.p[3], log(w), poly);
  const double r = phi * 0.31830988618379067;  // phi / pi
  return (float)(r - rint(r));
}

// u = h_+ + i h_x = v^2 exp(2 i phi) on the circular grid: sample j holds
// m = n - j samples before coalescence.  Grid (n / 256, templates).
__global__ __launch_bounds__(256) void k_td_gen(const SegDev* __restrict__ sd,
                                                const ci_tdparams* __restrict__ tdp,
                                                float2* __restrict__ u) {
  const int b = blockIdx.y;
  const int64_t n = sd->n;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const ci_tdparams& T = tdp[b];
  const int64_t m = n - j;
  float2 o = make_float2(0.f, 0.f);
  if (!(T.flags & CI_TMPL_EMPTY) && m >= T.m_lo && m <= T.m_hi) {
    const double w = td_solve_w(T, -(double)m / sd->fs);
    const float fr = td_phase_frac(T, w);
    const float a = __builtin_amdgcn_rcpf((float)(w * w));
    o = make_float2(a * __builtin_amdgcn_cosf(fr), a * __builtin_amdgcn_sinf(fr));
  }
  u[(size_t)b * n + j] = o;
}

// Split of the transform V = IDFT(h_+ + i h_x) of two real signals into
// theirs: Vp_k = (V_k + conj V_{n-k}) / 2 = IDFT(h_+)_k and
// Vc_k = (V_k - conj V_{n-k}) / (2i) = IDFT(h_x)_k.
__device__ __forceinline__ void td_split(float2 va, float2 vb, float2& vp, float2& vc) {
  vp = make_float2(0.5f * (va.x + vb.x), 0.5f * (va.y - vb.y));
  vc = make_float2(0.5f * (va.y + vb.y), 0.5f * (vb.x - va.x));
}

// Partial sums of S_+ = sum_band |Vp_k|^2 / S_k and S_x (likewise) over
// kTdChunks equal slices of the band, in FP64.  Grid (kTdChunks, templates).
__global__ __launch_bounds__(256) void k_td_sigma(const SegDev* __restrict__ sd,
                                                  const ci_tdparams* __restrict__ tdp,
                                                  const float2* __restrict__ V,
                                                  const double* __restrict__ isp,
                                                  double* __restrict__ sig) {
  __shared__ double sh[2][4];
  const int b = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
  const int64_t n = sd->n, half = sd->half;
  const int64_t kl = tdp[b].k_low;
  const int64_t len = half > kl ? half - kl : 0;
  const int64_t c0 = kl + len * ch / kTdChunks, c1 = kl + len * (ch + 1) / kTdChunks;
  const float2* vb = V + (size_t)b * n;
  double sp = 0.0, sc = 0.0;
  for (int64_t k = c0 + tid; k < c1; k += 256) {
    float2 vp, vc;
    td_split(vb[k], vb[n - k], vp, vc);
    const double w = isp[k];
    sp += ((double)vp.x * vp.x + (double)vp.y * vp.y) * w;
    sc += ((double)vc.x * vc.x + (double)vc.y * vc.y) * w;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sp += __shfl_xor(sp, off, 64);
    sc += __shfl_xor(sc, off, 64);
  }
  if ((tid & 63) == 0) {
    sh[0][tid >> 6] = sp;
    sh[1][tid >> 6] = sc;
  }
  __syncthreads();
  if (tid == 0) {
    sig[((size_t)b * kTdChunks + ch) * 2] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    sig[((size_t)b * kTdChunks + ch) * 2 + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
  }
}

// Spectra H~+_k = dt conj(Vp_k), H~x_k = dt conj(Vc_k) for k = 0..n/2 and
// sigma^2 = 4 df dt^2 S.  Grid (ceil((n/2 + 1) / 256), templates).
__global__ __launch_bounds__(256) void k_td_export(const SegDev* __restrict__ sd,
                                                   const float2* __restrict__ V,
                                                   const double* __restrict__ sig,
                                                   float2* __restrict__ hf,
                                                   double* __restrict__ sigma2) {
  const int b = blockIdx.y;
  const int64_t n = sd->n, m = sd->half + 1;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double dt = 1.0 / sd->fs;
  const float2* vb = V + (size_t)b * n;
  if (hf && k < m) {
    float2 vp, vc;
    td_split(vb[k], vb[(n - k) & (n - 1)], vp, vc);
    float2* o = hf + (size_t)b * 2 * m;
    o[k] = make_float2((float)(dt * vp.x), (float)(-dt * vp.y));
    o[m + k] = make_float2((float)(dt * vc.x), (float)(-dt * vc.y));
  }
  if (sigma2 && blockIdx.x == 0 && threadIdx.x < 2) {
    double s = 0.0;
    for (int i = 0; i < kTdChunks; ++i) s += sig[((size_t)b * kTdChunks + i) * 2 + threadIdx.x];
    sigma2[(size_t)b * 2 + threadIdx.x] = 4.0 * sd->df * dt * dt * s;
  }
}

struct P1Args {
  const ci_tparams* prm;   // batch's first template
  const float2* w;         // weighted data spectrum [n/2]
  const float2* tw;        // exp(2 pi i e / 2048)
  const float2* twa;       // exp(2 pi i e / n), e < 2048
  const float2* twb;       // exp(2 pi i 2048 e / n)
  const double2* tw64;     // exp(2 pi i e / 2048) in FP64
  float2* y;               // intermediate, [nb][n] in tile layout
  // per-batch trigger state to clear (null when not searching)
  u64* wkeys;
  int64_t nzero_w;         // entries of wkeys to clear
  u64* mkey;               // the batch's merge keys [nwin] (cleared too)
  int nwin;
  int nb;
  // two-polarization templates (k_pass1_mem)
  const float2* uv;        // [nb][n] spectrum in memory, natural order
  const ci_tdparams* tdp;  // batch's first template
  const float2* w0;        // g x~_k / S_k  [n/2]
  const double* sig;       // [nb][kTdChunks][2] sigma^2 partial sums
  const SegDev* sd;        // df and the data scale g of w0
};

// Packed FP16 storage of the intermediate (split-precision paths): one
// 32-bit word per complex value, real part in the low half.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned f2h(float2 v) {
  h2v h;
  h.x = (_Float16)v.x;
  h.y = (_Float16)v.y;
  return __builtin_bit_cast(unsigned, h);
}
__device__ __forceinline__ float2 h2f(unsigned u) {
  const h2v h = __builtin_bit_cast(h2v, u);
  return make_float2((float)h.x, (float)h.y);
}
__device__ __forceinline__ float2 ld_y(const float2* p, size_t i) { return p[i]; }
__device__ __forceinline__ float2 ld_y(const unsigned* p, size_t i) { return h2f(p[i]); }

// The intermediate is written once by pass 1 and read once by pass 2, and a
// batch of it (0.5-2 GiB) outlasts every cache: its stores are
// non-temporal, so they do not displace the cached spectrum and tables, and
// so are the 8-byte loads of the FP32 intermediate (measured: +8 % for the
// FP32 search; non-temporal 4-byte loads of the FP16 intermediate were
// slower, so those stay ordinary).
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ void st_nt(unsigned* p, unsigned v) { __builtin_nontemporal_store(v, p); }
typedef float f4s __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_nt16(float2* p, f4s v) {
  __builtin_nontemporal_store(v, reinterpret_cast<f4s*>(p));
}
__device__ __forceinline__ float2 ld_nt(const float2* p) {
  return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ unsigned ld_nt(const unsigned* p) { return *p; }

// Raw buffer descriptor of `bytes` bytes from p (gfx9 family: no swizzle,
// 32-bit data format).  Buffer loads take the address as a descriptor held
// in scalar registers plus a per-lane offset plus a scalar offset, so loads
// whose lanes keep fixed offsets from a common base need no vector address
// arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// 8 bytes at voff + soff (non-temporal) and 4 bytes at voff + soff.
__device__ __forceinline__ float2 buf_ld_nt(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 2));
}
__device__ __forceinline__ unsigned buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
// 16 bytes at voff + soff (non-temporal).
__device__ __forceinline__ f4s buf_ld16_nt(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(f4s, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 2));
}

// w_N^e for 0 <= e < N from the two-level table.
__device__ __forceinline__ float2 tw_n(const float2* __restrict__ twa,
                                       const float2* __restrict__ twb, int e) {
  return cmul(twa[e & 2047], twb[e >> 11]);
}

// Inputs of pass 1: Z_k of the frequency-domain chirp, generated on chip
// (zero outside the band).
struct SrcSpa {
  const ci_tparams& P;
  const float2* __restrict__ w;
  __device__ __forceinline__ float2 operator()(int k) const {
    float2 v = make_float2(0.f, 0.f);
    if (k >= P.k_low && k <= P.k_high) {
      const float2 e = chirp_phasor(P, k);
      v = cmul(w[k], make_float2(e.x * P.scale, e.y * P.scale));
    }
    return v;
  }
};

// Output forms of the first pass: FP16 pairs (one 4-byte store per value),
// FP32 (one 8-byte store per value) and FP32 in 16-byte stores of two
// columns' values.
enum P1Out { kOutF16 = 0, kOutF32 = 1, kOutF32Pair = 2 };

// Lane (c, t) of a first-pass workgroup of C N2 / 16 threads.  Paired FP32
// output: columns c and c + 1 (c even) sit 16 lanes apart in one wave (lane
// bit 4 is the low bit of c), so that the store can pair them with one row
// swap; each half wave still covers C consecutive columns of 32 / C
// consecutive rows, as with the columns in lane order, so its LDS and
// memory accesses touch the same addresses together.  Otherwise the
// columns in lane order: 4-byte FP16 stores lose their coalescing when
// neighbouring lanes hold alternate columns, and so do the scattered 8-byte
// loads of the two-polarization correlator.  Returned as values (through
// out-parameters the FP16 pass lost its stores' constant offsets: 99
// registers instead of 75).
template <int C, int OUT>
__device__ __forceinline__ unsigned p1_col(unsigned tid) {
  if constexpr (OUT != kOutF32Pair) return tid % C;
  const unsigned l = tid & 63u;
  return 2u * (l % (C / 2)) + ((l >> 4) & 1u);
}
template <int C, int OUT>
__device__ __forceinline__ unsigned p1_row(unsigned tid) {
  if constexpr (OUT != kOutF32Pair) return tid / C;
  const unsigned l = tid & 63u;
  return (tid >> 6) * (64u / C) + (l >> 5) * (32u / C) + (l & 15u) / (C / 2);
}

// Pass-1 body for one tile.  Q: number of stage-1 inputs per lane that can
// be nonzero (m < Q), chosen per template from its upper band edge.
// src(k) gives the input Z_k.
template <int N1, int N2, int C, int Q, int OUT, class Src>
__device__ __forceinline__ void pass1_tile(const P1Args& a, const Src& src, int b, int tile,
                                           float2* lds, const float2* twl, unsigned t,
                                           unsigned c) {
  using K = Col<N2, C>;
  constexpr int N = N1 * N2;
  constexpr int Lp = K::Lp;
  constexpr int R3 = K::R3;
  const unsigned k1 = tile * C + c;

  // Per-lane twiddle constants, read first so that their latency overlaps
  // the generation: the stage-2 twiddle merged with the four-step twiddle
  // w_N^{k1 j2} is base * w^{a2} (a geometric sequence in the stage-2
  // output a2), the radix-R3 outputs b add v^b.
  float2 base, w, v3 = make_float2(1.f, 0.f);
  if constexpr (R3 == 1) {
    // j2 = t + 16 a2 is final after stage 2
    base = tw_n(a.twa, a.twb, (int)(k1 * t));
    w = tw_n(a.twa, a.twb, (int)(16 * k1));
  } else {
    // rows d = a0 + 16 a2 of the radix-R3 step; output b adds 256 b to j2
    const unsigned a0 = t / R3, s2 = t % R3;
    base = tw_n(a.twa, a.twb, (int)(k1 * a0));
    w = cmul(twl[s2 * (N2 / (16 * R3))], tw_n(a.twa, a.twb, (int)(16 * k1)));
    v3 = tw_n(a.twa, a.twb, (int)(256 * k1));
  }

  // Z_k for k = k1 + N1 k2, k2 = t + Lp m.
  float2 x[16];
#pragma unroll
  for (int m = 0; m < Q; ++m) x[m] = src((int)(k1 + N1 * (t + Lp * m)));

  K::template stage1<Q, 1>(x, lds, t, c, twl);
  K::stage2(x, lds, t, c);
  x[0] = cmul(x[0], base);
#pragma unroll
  for (int a2 = 1; a2 < 16; ++a2) {
    base = cmul(base, w);
    x[a2] = cmul(x[a2], base);
  }
  K::stage3(x, lds, t, c);
  if constexpr (R3 > 1) {
    const float2 v = v3;
    float2 vb = v;
#pragma unroll
    for (int bb = 1; bb < R3; ++bb) {
#pragma unroll
      for (int i = 0; i < 16 / R3; ++i) x[i * R3 + bb] = cmul(x[i * R3 + bb], vb);
      vb = cmul(vb, v);
    }
  }

  const unsigned o = t * C + c;
  if constexpr (OUT == kOutF16) {
    unsigned* yt = reinterpret_cast<unsigned*>(a.y) + (size_t)b * N + (size_t)tile * N2 * C;
#pragma unroll
    for (int r = 0; r < 16; ++r) st_nt(&yt[o + K::off(r) * C], f2h(x[r]));
  } else if constexpr (OUT == kOutF32) {
    float2* yt = a.y + (size_t)b * N + (size_t)tile * N2 * C;
#pragma unroll
    for (int r = 0; r < 16; ++r) st_nt(&yt[o + K::off(r) * C], x[r]);
  } else {
    // Registers r and r + 1 hold rows off(r) and off(r) + D.  One row swap
    // per component (lanes as p1_col and p1_row place them) gives the lane of the
    // even column both columns' values of row off(r), and the lane 16 above
    // it (the odd column) both of row off(r + 1): each stores 16 bytes
    // (measured: pass 1 ~3 % faster than one 8-byte store per value).
    constexpr int D = K::off(1) - K::off(0);
    float2* yt = a.y + (size_t)b * N + (size_t)tile * N2 * C;
    float2* pb = yt + (o & ~1u) + ((c & 1u) ? D * C : 0);
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const auto re = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[r].x),
                                                       __float_as_uint(x[r + 1].x), false, false);
      const auto im = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[r].y),
                                                       __float_as_uint(x[r + 1].y), false, false);
      f4s v;
      v.x = __uint_as_float(re[0]);
      v.y = __uint_as_float(im[0]);
      v.z = __uint_as_float(re[1]);
      v.w = __uint_as_float(im[1]);
      st_nt16(pb + K::off(r) * C, v);
    }
  }
}

// H: store the intermediate as FP16 pairs (split-precision paths).
template <int N1, int N2, int C, bool H>
__global__ __launch_bounds__(C * N2 / 16) void k_pass1(P1Args a) {
  constexpr int Lp = N2 / 16;
  constexpr int TILES = N1 / C;
  extern __shared__ float2 lds[];
  const unsigned tid = threadIdx.x;
  constexpr int OUT = H ? kOutF16 : kOutF32Pair;
  const unsigned c = p1_col<C, OUT>(tid), t = p1_row<C, OUT>(tid);

  if (a.wkeys) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + tid;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gid; i < a.nzero_w; i += gsz) a.wkeys[i] = 0ull;
    for (int64_t i = gid; i < a.nwin; i += gsz) a.mkey[i] = 0ull;
  }

  // w_{N2}^e, e < N2, in LDS after the exchange buffer (stage-1 and
  // stage-2 twiddles)
  float2* twl = lds + Col<N2, C>::LDS_ELEMS;
  for (int k = (int)tid; k < N2; k += (int)blockDim.x) twl[k] = a.tw[k * (2048 / N2)];
  __syncthreads();

  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int b = bid / TILES, tile = bid % TILES;
  const ci_tparams P = a.prm[b];
  // Every band bin lies below n/2 (k2 < N2/2, so m < 8), and below k_high:
  // m <= (k_high / N1) / Lp.  The choice is uniform over the workgroup.
  const int mneed = P.k_high >= P.k_low ? (P.k_high / N1) / Lp + 1 : 1;
  const SrcSpa src{P, a.w};
  if (mneed <= 2) pass1_tile<N1, N2, C, 2, OUT>(a, src, b, tile, lds, twl, t, c);
  else if (mneed <= 4) pass1_tile<N1, N2, C, 4, OUT>(a, src, b, tile, lds, twl, t, c);
  else pass1_tile<N1, N2, C, 8, OUT>(a, src, b, tile, lds, twl, t, c);
}

// ---------------------------------------------------------------------------
// two-polarization time-domain templates
// ---------------------------------------------------------------------------

// Input of the plain inverse DFT of a spectrum held in memory.
struct SrcMem {
  const float2* __restrict__ z;
  __device__ __forceinline__ float2 operator()(int k) const { return z[k]; }
};

// Input of the two-polarization correlator transform.  For a real template
// IDFT(h)_k = conj(H~_k) / dt, so with a_k = ap w0_k Vp_k and
// b_k = ac w0_k Vc_k (ap = sqrt(4 df / S_+) / (2 g), S_+ = sum_band
// |Vp_k|^2 / S_k, likewise ac) the band bins carry (a_k + i b_k) and their
// mirrors n - k carry conj(a_k) + i conj(b_k): the inverse DFT of that
// packed spectrum is c_+ + i c_x, the paper's two C2R outputs at once.
struct SrcTd {
  const float2* __restrict__ V;
  const float2* __restrict__ w0;
  float ap, ac;
  int k_low, half, n;
  __device__ __forceinline__ float2 operator()(int k) const {
    int kk;
    bool mir;
    if (k >= k_low && k < half) {
      kk = k;
      mir = false;
    } else if (k > half && n - k >= k_low) {
      kk = n - k;
      mir = true;
    } else {
      return make_float2(0.f, 0.f);
    }
    float2 vp, vc;
    td_split(V[kk], V[n - kk], vp, vc);
    const float2 x = w0[kk];
    const float2 pa = cmul(x, vp), pb = cmul(x, vc);
    const float2 av = make_float2(pa.x * ap, pa.y * ap);
    const float2 bv = make_float2(pb.x * ac, pb.y * ac);
    return mir ? make_float2(av.x + bv.y, bv.x - av.y) : make_float2(av.x - bv.y, av.y + bv.x);
  }
};

// Input of the template transform generated on the fly: the sample
// u_j = h_+ + i h_x of a two-polarization template (as k_td_gen writes it).
struct SrcGen {
  const ci_tdparams& T;
  int64_t n;
  double fs;
  __device__ __forceinline__ float2 operator()(int j) const {
    const int64_t m = n - j;
    if ((T.flags & CI_TMPL_EMPTY) || m < T.m_lo || m > T.m_hi) return make_float2(0.f, 0.f);
    const double w = td_solve_w(T, -(double)m / fs);
    const float fr = td_phase_frac(T, w);
    const float a = __builtin_amdgcn_rcpf((float)(w * w));
    return make_float2(a * __builtin_amdgcn_cosf(fr), a * __builtin_amdgcn_sinf(fr));
  }
};

// Pass 1 over a spectrum held in memory, every bin possibly nonzero.
// MODE 0: the plain inverse DFT of a.uv.  MODE 1: the two-polarization
// correlator built from a.uv = IDFT(h_+ + i h_x) and w0.  MODE 2: the
// inverse DFT of u = h_+ + i h_x generated on the fly (no u in memory).
template <int N1, int N2, int C, int MODE>
__global__ __launch_bounds__(C * N2 / 16) void k_pass1_mem(P1Args a) {
  constexpr int N = N1 * N2;
  constexpr int TILES = N1 / C;
  extern __shared__ float2 lds[];
  const unsigned tid = threadIdx.x;
  // the correlator (MODE 1) reads three scattered values per bin: columns
  // in lane order, 8-byte stores
  constexpr int OUT = MODE == 1 ? kOutF32 : kOutF32Pair;
  const unsigned c = p1_col<C, OUT>(tid), t = p1_row<C, OUT>(tid);

  if (a.wkeys) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + tid;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gid; i < a.nzero_w; i += gsz) a.wkeys[i] = 0ull;
    for (int64_t i = gid; i < a.nwin; i += gsz) a.mkey[i] = 0ull;
  }
  float2* twl = lds + Col<N2, C>::LDS_ELEMS;
  for (int k = (int)tid; k < N2; k += (int)blockDim.x) twl[k] = a.tw[k * (2048 / N2)];
  __syncthreads();

  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int b = bid / TILES;
  int tile = bid % TILES;
  if constexpr (MODE == 1) {
    // The correlator reads each bin k and its mirror n - k, which lies in
    // column N1 - k1: tiles m and TILES - 1 - m run next to each other on
    // one XCD, so that the second read of a value can find it in that XCD's
    // L2 (measured: the pass 5 % faster, though most values are still
    // fetched twice).
    const int i = tile;
    tile = (i & 1) ? TILES - 1 - (i >> 1) : (i >> 1);
  }
  const float2* vb = a.uv + (size_t)b * N;
  if constexpr (MODE == 0) {
    pass1_tile<N1, N2, C, 16, OUT>(a, SrcMem{vb}, b, tile, lds, twl, t, c);
  } else if constexpr (MODE == 2) {
    const ci_tdparams& T = a.tdp[b];
    pass1_tile<N1, N2, C, 16, OUT>(a, SrcGen{T, (int64_t)N, a.sd->fs}, b, tile, lds, twl, t,
                                     c);
  } else {
    // sigma^2 sums in a fixed order
    const double* sg = a.sig + (size_t)b * kTdChunks * 2;
    double sp = 0.0, sc = 0.0;
    for (int i = 0; i < kTdChunks; ++i) {
      sp += sg[2 * i];
      sc += sg[2 * i + 1];
    }
    const ci_tdparams& T = a.tdp[b];
    const bool live = !(T.flags & CI_TMPL_EMPTY) && sp > 0.0 && sc > 0.0;
    const double df = a.sd->df, g = a.sd->g;
    const float ap = live ? (float)(0.5 * sqrt(4.0 * df / sp) / g) : 0.f;
    const float ac = live ? (float)(0.5 * sqrt(4.0 * df / sc) / g) : 0.f;
    const SrcTd src{vb, a.w0, ap, ac, T.k_low, N / 2, N};
    pass1_tile<N1, N2, C, 16, OUT>(a, src, b, tile, lds, twl, t, c);
  }
}

// ---------------------------------------------------------------------------
// pass 2 helpers
// ---------------------------------------------------------------------------

// Load the pass-2 column inputs: lane (cc, t) of tile `tile` gets
// x[q] = Y[k1 = t + (N1/16) q][j2 = tile J + cc].
template <int N1, int N2, int C, int J>
__device__ __forceinline__ void load_pass2(float2 (&x)[16], const float2* __restrict__ yb,
                                           unsigned j2, unsigned t) {
  constexpr unsigned Lp = N1 / 16;
  static_assert(Lp % C == 0, "tile width divides the stage stride");
  const float2* p = yb + ((t / C) * N2 + j2) * C + (t % C);
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = ld_nt(&p[q * (Lp * N2)]);
}


template <int N1, int N2, int C, int J>
__device__ __forceinline__ void load_pass2(float2 (&x)[16], const unsigned* __restrict__ yb,
                                           unsigned j2, unsigned t) {
  constexpr unsigned Lp = N1 / 16;
  const unsigned* p = yb + ((t / C) * N2 + j2) * C + (t % C);
  unsigned u[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) u[q] = ld_nt(&p[q * (Lp * N2)]);
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = h2f(u[q]);
}

// z_j = sum_{k1} exp(2 pi i j1 k1 / N1) Y[k1][j2] for j = j2 + N2 j1, with
// FP64 twiddles and accumulation, computed by one wave (64 lanes, N1/64
// terms each, then a butterfly reduction); every lane returns the result.
template <int N1, int N2, int C, typename T>
__device__ double2 wave_direct_z(const T* __restrict__ yb, const double2* __restrict__ tw64,
                                 int64_t j) {
  const int lane = threadIdx.x & 63;
  const int j2 = (int)(j % N2), j1 = (int)(j / N2);
  constexpr int PER = N1 / 64;
  float2 v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int k1 = lane + 64 * i;
    v[i] = ld_y(yb, ((size_t)(k1 / C) * N2 + j2) * C + (k1 % C));
  }
  double re = 0.0, im = 0.0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int k1 = lane + 64 * i;
    const int e = (int)(((int64_t)j1 * k1) % N1);
    const double2 w = tw64[e * (2048 / N1)];
    re += (double)v[i].x * w.x - (double)v[i].y * w.y;
    im += (double)v[i].x * w.y + (double)v[i].y * w.x;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  return make_double2(re, im);
}

// Wave-wide maximum / minimum through data-parallel-primitive lane moves
// (no LDS round trips): pairs, quads, 8- and 16-lane mirrors within each
// row of 16 lanes, then the row broadcasts carry each row's result into the
// next rows; lane 63 ends with the wave's value, which is read back to every
// lane.  Lanes a move cannot source keep their own value.
template <typename T, typename F>
__device__ __forceinline__ T wave_reduce(T v, F op) {
  int x = __builtin_bit_cast(int, v);
  x = __builtin_bit_cast(int, op(__builtin_bit_cast(T, x), __builtin_bit_cast(T,
                         __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false))));   // quad_perm 1,0,3,2
  x = __builtin_bit_cast(int, op(__builtin_bit_cast(T, x), __builtin_bit_cast(T,
                         __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false))));   // quad_perm 2,3,0,1
  x = __builtin_bit_cast(int, op(__builtin_bit_cast(T, x), __builtin_bit_cast(T,
                         __builtin_amdgcn_update_dpp(x, x, 0x141, 0xF, 0xF, false))));  // row_half_mirror
  x = __builtin_bit_cast(int, op(__builtin_bit_cast(T, x), __builtin_bit_cast(T,
                         __builtin_amdgcn_update_dpp(x, x, 0x140, 0xF, 0xF, false))));  // row_mirror
  x = __builtin_bit_cast(int, op(__builtin_bit_cast(T, x), __builtin_bit_cast(T,
                         __builtin_amdgcn_update_dpp(x, x, 0x142, 0xA, 0xF, false))));  // row_bcast:15
  x = __builtin_bit_cast(int, op(__builtin_bit_cast(T, x), __builtin_bit_cast(T,
                         __builtin_amdgcn_update_dpp(x, x, 0x143, 0xC, 0xF, false))));  // row_bcast:31
  return __builtin_bit_cast(T, __builtin_amdgcn_readlane(x, 63));
}

__device__ __forceinline__ float wave_max(float v) {
  return wave_reduce(v, [](float a, float b) { return fmaxf(a, b); });
}
__device__ __forceinline__ unsigned wave_min(unsigned v) {
  return wave_reduce(v, [](unsigned a, unsigned b) { return a < b ? a : b; });
}

__device__ __forceinline__ u64 aload(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of one int per lane over the workgroup (Hillis-Steele in
// LDS).  Returns the exclusive prefix; *total receives the sum.
__device__ int block_excl_scan(int v, int* sh, int* total) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __syncthreads();
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const int u = (tid >= off) ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += u;
    __syncthreads();
  }
  const int incl = sh[tid];
  *total = sh[nt - 1];
  __syncthreads();
  return incl - v;
}

struct P2Args {
  const char* flagp;         // flags of the batch's first template ...
  int flag_stride;           // ... and the byte stride to the next one
  const float2* tw;
  const double2* tw64;
  const float2* y;           // intermediate of this batch
  int64_t t0;                // bank index of the batch's first template
  int nb;
  // trigger mode
  u64* ppart;                // [nb][ntile2] peak keys of the second pass
  int ntile2;                // peak keys per template: one per workgroup, or
                             // one per wave with wave-owned columns
  u64* wkeys;                // [nb][nwin]
  u64* mkey;                 // [nwin] per window: max over the batch of
                             // (rho^2 bits, complemented template index)
  int* cnt;                  // [nb]
  int* sidx;                 // [nb][nwin]
  ci_trigger* stage;         // [nb][nwin]
  ci_trigger* mrec;          // [nwin]
  u64* run;                  // [1]
  int nwin;
  int64_t window;
  int64_t j_lo, j_hi;
  int jlo32, jhi32, full;    // the same range as int32, and whether it is [0, n)
  unsigned int win32;        // window as uint32
  float thr2;
  ci_trigger* d_peaks;       // whole bank
  ci_trigger* d_trig;
  int64_t cap;
  int64_t* d_count;
  int merge;
  int last_batch;
  // series mode
  float2* z;                 // batch's first series
  int half_y;                // intermediate stored as packed FP16 pairs
  const uint4* mxa;          // matrix-core fragments of the pass-2 column DFT
};

// Peak and triggers of template b once all its pass-2 tiles are done: the
// peak key is the max of the tiles' partials; the windows with a key are
// compacted in window order; z at the peak and at every trigger is
// recomputed from the intermediate, one sample per wave at a time.
template <int N1, int N2, int C>
__device__ void finalize_template(const P2Args& a, int b, void* ldsv) {
  constexpr int N = N1 * N2;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63, nwaves = nt >> 6;
  int* iscr = reinterpret_cast<int*>(ldsv);
  const int32_t flags = *reinterpret_cast<const int32_t*>(a.flagp + (size_t)b * a.flag_stride);
  const int64_t tg = a.t0 + b;
  const float2* yb = a.y + (size_t)b * N;
  // peak key: max over the pass-2 workgroups' partials
  u64 pk = 0ull;
  for (int i = tid; i < a.ntile2; i += nt) {
    const u64 v = a.ppart[(size_t)b * a.ntile2 + i];
    pk = v > pk ? v : pk;
  }
  {
    u64* ush = reinterpret_cast<u64*>(ldsv);
    __syncthreads();
    ush[tid] = pk;
    __syncthreads();
    for (int off = nt / 2; off > 0; off >>= 1) {
      if (tid < off) ush[tid] = ush[tid + off] > ush[tid] ? ush[tid + off] : ush[tid];
      __syncthreads();
    }
    pk = ush[0];
    __syncthreads();
  }
  if ((flags & CI_TMPL_EMPTY) || pk == 0ull) {
    if (tid == 0) {
      ci_trigger e;
      e.tmpl = tg; e.index = -1; e.rho2 = 0.f; e.re = 0.f; e.im = 0.f; e.window = -1;
      a.d_peaks[tg] = e;
      a.cnt[b] = 0;
    }
    return;
  }
  // compact the windows whose key is set, in window order
  const u64* wk = a.wkeys + (size_t)b * a.nwin;
  const int per = (a.nwin + nt - 1) / nt;
  const int w0 = tid * per;
  const int w1 = min(w0 + per, a.nwin);
  int mine = 0;
  for (int w = w0; w < w1; ++w) mine += (aload(&wk[w]) != 0ull);
  int total = 0;
  if (__syncthreads_or(mine) != 0) {
    int pos = block_excl_scan(mine, iscr, &total);
    ci_trigger* st = a.stage + (size_t)b * a.nwin;
    int* sx = a.sidx + (size_t)b * a.nwin;
    for (int w = w0; w < w1; ++w) {
      const u64 key = aload(&wk[w]);
      if (key != 0ull) {
        ci_trigger e;
        e.tmpl = tg;
        e.index = (int64_t)(0xFFFFFFFFu - (unsigned int)(key & 0xFFFFFFFFull));
        e.rho2 = __uint_as_float((unsigned int)(key >> 32));
        e.re = 0.f; e.im = 0.f; e.window = w;
        st[pos] = e;
        sx[w] = pos;
        ++pos;
        // the batch's best template per window (larger rho^2; ties to the
        // smaller template), for the merge
        if (a.merge)
          atomicMax(&a.mkey[w], (key & 0xFFFFFFFF00000000ull) | (u64)(0xFFFFFFFFu - (unsigned)b));
      }
    }
    __syncthreads();
  }
  // item 0: the peak; items 1..total: the triggers, one wave per item
  ci_trigger* st = a.stage + (size_t)b * a.nwin;
  for (int it = wave; it <= total; it += nwaves) {
    const int64_t j = it == 0 ? (int64_t)(0xFFFFFFFFu - (unsigned int)(pk & 0xFFFFFFFFull))
                              : st[it - 1].index;
    const double2 z =
        a.half_y ? wave_direct_z<N1, N2, C>(reinterpret_cast<const unsigned*>(a.y) + (size_t)b * N,
                                            a.tw64, j)
                 : wave_direct_z<N1, N2, C>(yb, a.tw64, j);
    if (lane == 0) {
      if (it == 0) {
        ci_trigger e;
        e.tmpl = tg; e.index = j; e.rho2 = __uint_as_float((unsigned int)(pk >> 32));
        e.re = (float)z.x; e.im = (float)z.y; e.window = (int)(j / a.window);
        a.d_peaks[tg] = e;
      } else {
        st[it - 1].re = (float)z.x;
        st[it - 1].im = (float)z.y;
      }
    }
  }
  if (tid == 0) a.cnt[b] = total;
}

// Place the batch's triggers into the caller's list (or merge them), once
// every template of the batch is finalised.
__device__ void place_batch(const P2Args& a, void* ldsv) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int* iscr = reinterpret_cast<int*>(ldsv);
  if (!a.merge) {
    // offsets in template order: each lane sums a run of templates, one
    // workgroup scan over the runs
    __shared__ long long s_base;
    if (tid == 0) s_base = (long long)a.run[0];
    const int per = (a.nb + nt - 1) / nt;
    const int b0 = tid * per, b1 = min(b0 + per, a.nb);
    int mine = 0;
    for (int b = b0; b < b1; ++b) mine += a.cnt[b];
    int total = 0;
    int off = block_excl_scan(mine, iscr, &total);
    const long long base = s_base;
    for (int b = b0; b < b1; ++b) {
      const int c = a.cnt[b];
      const ci_trigger* st = a.stage + (size_t)b * a.nwin;
      for (int i = 0; i < c; ++i) {
        const long long p = base + off + i;
        if (p < a.cap) a.d_trig[p] = st[i];
      }
      off += c;
    }
    if (tid == 0) {
      a.run[0] = (u64)(base + total);
      a.d_count[0] = base + total;
    }
    return;
  }
  // merge: per window, largest rho^2 over templates, earlier template wins
  // ties (within the batch through the merge key, across batches because
  // a later batch must be strictly larger)
  for (int w = tid; w < a.nwin; w += nt) {
    const u64 key = aload(&a.mkey[w]);
    if (key == 0ull) continue;
    const int b = (int)(0xFFFFFFFFu - (unsigned int)(key & 0xFFFFFFFFull));
    const float r2 = __uint_as_float((unsigned int)(key >> 32));
    const ci_trigger best = a.mrec[w];
    if (best.tmpl < 0 || r2 > best.rho2)
      a.mrec[w] = a.stage[(size_t)b * a.nwin + a.sidx[(size_t)b * a.nwin + w]];
  }
  if (!a.last_batch) return;
  __syncthreads();
  // compact the merged records in window order
  const int per = (a.nwin + nt - 1) / nt;
  const int w0 = tid * per;
  const int w1 = min(w0 + per, a.nwin);
  int mine = 0;
  for (int w = w0; w < w1; ++w) mine += (a.mrec[w].tmpl >= 0);
  int total = 0;
  int pos = block_excl_scan(mine, iscr, &total);
  for (int w = w0; w < w1; ++w) {
    if (a.mrec[w].tmpl >= 0) {
      if (pos < a.cap) a.d_trig[pos] = a.mrec[w];
      ++pos;
    }
  }
  if (tid == 0) a.d_count[0] = total;
}

// ---------------------------------------------------------------------------
// pass 2: second four-step pass + post-pass
// ---------------------------------------------------------------------------

// Byte offset of lane (cc, t)'s first pass-2 input, Y[k1 = t][j2 = cc],
// from a tile's first column: the same for every tile.
template <int N1, int N2, int C>
__device__ __forceinline__ unsigned p2_lane_off(unsigned cc, unsigned t) {
  return (((t / C) * N2 + cc) * C + (t % C)) * (unsigned)sizeof(float2);
}

// x[q] = Y[k1 = t + (N1/16) q][j2 = tile J + cc] of pass-2 item `item`
// (as load_pass2), through a buffer descriptor at the tile's first column
// (the same for every lane), the lane's fixed offset voff = p2_lane_off(cc,
// t) and the constant offset of q.
template <int N1, int N2, int C, int J>
__device__ __forceinline__ void load_item(float2 (&x)[16], const P2Args& a, int item,
                                          unsigned voff) {
  constexpr int N = N1 * N2;
  constexpr int TILES = N2 / J;
  constexpr unsigned QS = (N1 / 16) * N2 * (unsigned)sizeof(float2);
  const int b = item / TILES, tile = item % TILES;
  const unsigned first = (unsigned)tile * J * C;
  const __amdgpu_buffer_rsrc_t r =
      buf_rsrc(a.y + (size_t)b * N + first, (N - first) * (unsigned)sizeof(float2));
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = buf_ld_nt(r, voff, q * QS);
}

// load_item in 16-byte loads, for lanes placed as in k_pass2w: the lane of
// row t (t even) loads rows t and t + 1 of register q, the lane 16 above it
// (row t + 1) the same two rows of register q + 1, q even; voff =
// p2_lane_off(cc, t & ~1) + (t & 1) QS.  The values stay as loaded, so that
// a prefetch does not wait for them; unpair_item hands each lane its own.
template <int N1, int N2, int C, int J>
__device__ __forceinline__ void load_item_pairs(f4s (&v)[8], const P2Args& a, int item,
                                                unsigned voff) {
  constexpr int N = N1 * N2;
  constexpr int TILES = N2 / J;
  constexpr unsigned QS = (N1 / 16) * N2 * (unsigned)sizeof(float2);
  const int b = item / TILES, tile = item % TILES;
  const unsigned first = (unsigned)tile * J * C;
  const __amdgpu_buffer_rsrc_t r =
      buf_rsrc(a.y + (size_t)b * N + first, (N - first) * (unsigned)sizeof(float2));
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = buf_ld16_nt(r, voff, 2 * i * QS);
}
// One row swap per component: the lane of row t keeps (t, q) and receives
// (t, q + 1); the lane of row t + 1 receives (t + 1, q) and keeps
// (t + 1, q + 1).
__device__ __forceinline__ void unpair_item(const f4s (&v)[8], float2 (&x)[16]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto re = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i].x),
                                                     __float_as_uint(v[i].z), false, false);
    const auto im = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i].y),
                                                     __float_as_uint(v[i].w), false, false);
    x[2 * i] = make_float2(__uint_as_float(re[0]), __uint_as_float(im[0]));
    x[2 * i + 1] = make_float2(__uint_as_float(re[1]), __uint_as_float(im[1]));
  }
}

// Post-pass of one pass-2 tile (workgroup of NW waves).  r2[i], i < K, are
// this lane's |z|^2 values (-1 outside the search range) in increasing
// sample index j = jof(i).  Samples above the threshold raise their
// window's key; the tile's peak key (rho^2 bits over the complemented
// smallest index with that value) goes to a.ppart[pidx].  The lane maximum
// decides both the threshold test and the peak; only lanes holding the
// workgroup maximum search for its index.
template <int K, int NW, typename JF>
__device__ __forceinline__ void tile_post(const float (&r2)[K], JF jof, const P2Args& a, int bt,
                                          size_t pidx, float* s_m, unsigned* s_j,
                                          unsigned tid) {
  const unsigned lane = tid & 63, wave = tid >> 6;
  float m = r2[0];
#pragma unroll
  for (int i = 1; i < K; ++i) m = fmaxf(m, r2[i]);
  if (__any(m > a.thr2)) {
    // rare: samples above threshold update their window's key
    u64* wk = a.wkeys + (size_t)bt * a.nwin;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (r2[i] > a.thr2) {
        const unsigned j = jof(i);
        const u64 key = ((u64)__float_as_uint(r2[i]) << 32) | (u64)(0xFFFFFFFFu - j);
        atomicMax(&wk[j / a.win32], key);
      }
    }
  }
  const float wm = wave_max(m);
  if (lane == 0) s_m[wave] = wm;
  __syncthreads();
  float M = s_m[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) M = fmaxf(M, s_m[w]);
  unsigned jm = 0xFFFFFFFFu;
  if (M >= 0.f && __any(m == M)) {
    if (m == M) {
#pragma unroll
      for (int i = K - 1; i >= 0; --i)
        if (r2[i] == M) jm = jof(i);
    }
    jm = wave_min(jm);
  }
  if (lane == 0) s_j[wave] = jm;
  __syncthreads();
  if (tid == 0) {
    unsigned j = s_j[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) j = min(j, s_j[w]);
    a.ppart[pidx] = M >= 0.f ? (((u64)__float_as_uint(M) << 32) | (u64)(0xFFFFFFFFu - j)) : 0ull;
  }
}

// Post-pass of the samples one wave holds (wave-owned columns): as
// tile_post, with the wave's peak key going to a.ppart[pidx] and no
// workgroup barrier, so the waves of a workgroup run independently.
template <int K, typename JF>
__device__ __forceinline__ void wave_post(const float (&r2)[K], JF jof, const P2Args& a, int bt,
                                          size_t pidx, unsigned lane) {
  float m = r2[0];
#pragma unroll
  for (int i = 1; i < K; ++i) m = fmaxf(m, r2[i]);
  if (__any(m > a.thr2)) {
    u64* wk = a.wkeys + (size_t)bt * a.nwin;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (r2[i] > a.thr2) {
        const unsigned j = jof(i);
        const u64 key = ((u64)__float_as_uint(r2[i]) << 32) | (u64)(0xFFFFFFFFu - j);
        atomicMax(&wk[j / a.win32], key);
      }
    }
  }
  const float M = wave_max(m);
  unsigned jm = 0xFFFFFFFFu;
  if (M >= 0.f && m == M) {
#pragma unroll
    for (int i = K - 1; i >= 0; --i)
      if (r2[i] == M) jm = jof(i);
  }
  jm = wave_min(jm);
  if (lane == 0)
    a.ppart[pidx] = M >= 0.f ? (((u64)__float_as_uint(M) << 32) | (u64)(0xFFFFFFFFu - jm)) : 0ull;
}

template <int N1, int N2, int C, int J>
__device__ __forceinline__ void pass2_post(const float2 (&x)[16], const P2Args& a, int b, int tile,
                                           u64* s_best, unsigned tid, unsigned cc, unsigned t);

// Second four-step pass and post-pass of one tile (J columns j2).
template <int N1, int N2, int C, int J>
__device__ __forceinline__ void pass2_tile(float2 (&x)[16], const P2Args& a, int item,
                                           float2* lds, const float2* twl, u64* s_best,
                                           unsigned tid, unsigned cc, unsigned t) {
  constexpr int TILES = N2 / J;
  const int b = item / TILES, tile = item % TILES;
  fft_col<N1, J, 1>(x, lds, t, cc, twl);
  pass2_post<N1, N2, C, J>(x, a, b, tile, s_best, tid, cc, t);
}

// Post-pass of one pass-2 tile: x holds z for j1 = Col::out(t, r) of column
// j2 = tile J + cc.
template <int N1, int N2, int C, int J>
__device__ __forceinline__ void pass2_post(const float2 (&x)[16], const P2Args& a, int b, int tile,
                                           u64* s_best, unsigned tid, unsigned cc, unsigned t) {
  constexpr int TILES = N2 / J;
  using K = Col<N1, J>;
  const unsigned j2 = tile * J + cc;
  auto jof = [&](int kk) { return j2 + (unsigned)N2 * (unsigned)K::out((int)t, K::reg_by_order(kk)); };
  float r2[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const float2 z = x[K::reg_by_order(kk)];
    r2[kk] = fmaf(z.x, z.x, z.y * z.y);
  }
  if (!a.full) {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int j = (int)jof(kk);
      if (j < a.jlo32 || j >= a.jhi32) r2[kk] = -1.f;
    }
  }
  float* s_m = reinterpret_cast<float*>(s_best);
  unsigned* s_j = reinterpret_cast<unsigned*>(s_best) + 16;
  tile_post<16, J * N1 / 16 / 64>(r2, jof, a, b, (size_t)b * TILES + tile, s_m, s_j, tid);
}

// Persistent pass 2: each workgroup walks tiles item = blockIdx.x + k G
// and prefetches the next tile's column inputs into registers while it
// transforms the current one, so that a CU keeps loads in flight during
// its butterflies.  Four waves per SIMD (at most 128 registers) except for
// 2048-point rows in workgroups of 512 threads, whose radix-8 stage and
// prefetch need more: two waves per SIMD there, so that nothing spills.
template <int N1, int N2, int C, int J>
__global__ __launch_bounds__(J * N1 / 16, (N1 >= 2048 && J * N1 / 16 <= 512) ? 2 : 4)
    void k_pass2_trig(P2Args a) {
  constexpr int TILES = N2 / J;
  using K = Col<N1, J>;
  extern __shared__ float2 lds[];
  __shared__ u64 s_best[16];
  const unsigned tid = threadIdx.x;
  const unsigned cc = tid % J, t = tid / J;
  const int total = a.nb * TILES;

  // w_{N1}^e, e < N1, copied once into LDS behind the exchange buffer: the
  // stage twiddles then never wait behind the prefetched tile's loads
  // (vector-memory loads retire in order).
  float2* twl = lds + K::LDS_ELEMS;
  for (unsigned e = tid; e < (unsigned)N1; e += blockDim.x) twl[e] = a.tw[e * (2048 / N1)];
  __syncthreads();

  const unsigned voff = p2_lane_off<N1, N2, C>(cc, t);
  float2 xn[16];
  const int G = gridDim.x;
  int item = blockIdx.x;
  if (item < total) load_item<N1, N2, C, J>(xn, a, item, voff);
  for (; item < total; item += G) {
    float2 x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = xn[r];
    if (item + G < total) load_item<N1, N2, C, J>(xn, a, item + G, voff);
    pass2_tile<N1, N2, C, J>(x, a, item, lds, twl, s_best, tid, cc, t);
  }
}

// Completion of this wave's LDS operations (the exchange rows are private
// to the wave, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// ---------------------------------------------------------------------------
// pass 2 with wave-owned columns after the first stage (FP32, N1 = 512 or
// 1024)
// ---------------------------------------------------------------------------
// The column DFT of k_pass2_trig with the same arithmetic in the same order,
// laid out so that only one exchange crosses waves.  Lanes load and run
// stage 1 on (column cc, row t) as there, with rows t and t + 1 placed 16
// lanes apart so that the intermediate is read in 16-byte loads (a wave's
// load covers the same whole runs of J x C contiguous elements as 8-byte
// loads in lane order, for two registers at once; measured: that pass ~3 %
// faster).  The exchange after stage 1 hands every
// column to Lp consecutive lanes of one wave (cb = tid / Lp, tb = tid %
// Lp); the exchange between stage 2 and the radix-R3 stage then stays
// inside the wave (its own column's LDS, no workgroup barrier), and the
// post-pass reduces per wave (one peak partial per wave).  Two workgroup
// barriers per tile instead of five.
// LDS: column-major exchange regions of X float2 per column.  Exchange 1
// stores (row a, position t) of column c at c X + a S1 + t; exchange 2
// stores (row d, position s) at c X + s RS + d.  The paddings make the
// stores and loads of each exchange touch distinct banks for 32
// consecutive lanes.
template <int N1, int J>
struct WaveCol {
  static constexpr int L = N1, Lp = L / 16, R3 = L / 256;
  static_assert(R3 == 2 || R3 == 4, "N1 = 512 or 1024");
  static_assert((J * Lp) % 64 == 0, "whole waves");
  static constexpr int S1 = Lp + R3;
  static constexpr int X = 16 * S1 + 32 / J;
  static constexpr int RS = L / R3 + 32 / R3;
  static_assert(R3 * RS <= X, "exchange 2 fits the column region");
  static constexpr int NW = J * Lp / 64;      // waves per workgroup
  static constexpr size_t lds_bytes() { return (size_t)(J * X + N1) * sizeof(float2); }
};

template <int N1, int N2, int C, int J>
__global__ __launch_bounds__(J * N1 / 16, 4) void k_pass2w(P2Args a) {
  using W = WaveCol<N1, J>;
  constexpr int Lp = W::Lp, R3 = W::R3, S1 = W::S1, X = W::X, RS = W::RS;
  constexpr int TILES = N2 / J;
  extern __shared__ float2 lds[];
  const unsigned tid = threadIdx.x;
  // load / stage-1 layout: column cc, row t, with rows t and t + 1 (t
  // even) 16 lanes apart in one wave and each half wave covering J
  // columns of 32 / J consecutive rows (as with the columns in lane order)
  const unsigned l64 = tid & 63u;
  const unsigned cc = l64 % J;
  const unsigned t = (tid >> 6) * (64u / J) + ((l64 >> 4) & 1u) +
                     2u * ((l64 / J) & (16u / J - 1u)) + (l64 >> 5) * (32u / J);
  const unsigned cb = tid / Lp, tb = tid % Lp;      // stage-2 / stage-3 layout
  const unsigned a0 = tb / R3, s2 = tb % R3;
  const unsigned lane = tid & 63, wave = tid >> 6;
  const int total = a.nb * TILES;

  // Twiddle tables behind the exchange regions, laid out so that a lane
  // reads every twiddle at a fixed offset from one base address:
  // t1[(q - 1) Lp + t] = w_L^{q t} (stage 1), t2[(a2 - 1) R3 + s2] =
  // w_L^{16 a2 s2} (stage 2), q, a2 = 1..15.
  float2* t1 = lds + J * X;
  float2* t2 = t1 + 15 * Lp;
  static_assert(15 * (Lp + R3) <= N1, "twiddle tables fit the reserved region");
  for (unsigned e = tid; e < 15u * (Lp + R3); e += blockDim.x) {
    unsigned x;
    if (e < 15u * Lp) x = (e / Lp + 1) * (e % Lp);
    else x = 16 * ((e - 15 * Lp) / R3 + 1) * ((e - 15 * Lp) % R3);
    t1[e] = a.tw[(x % N1) * (2048 / N1)];
  }
  __syncthreads();
  const float2* t1l = t1 + t;
  const float2* t2l = t2 + s2;

  auto tile_body = [&](float2 (&x)[16], int item) {
    const int b = item / TILES, tile = item % TILES;

    // stage 1: radix 16 over m, twiddle w_L^{a t}
    idft16(x);
#pragma unroll
    for (int q = 1; q < 16; ++q) x[q] = cmul(x[q], t1l[(q - 1) * Lp]);
    // exchange 1 (across waves): the previous tile's column regions are
    // free once every wave is past its exchange 2
    __syncthreads();
    {
      float2* pw = lds + cc * X + t;
#pragma unroll
      for (int q = 0; q < 16; ++q) pw[q * S1] = x[q];
    }
    __syncthreads();
    // stage 2: row a0, positions s2 + R3 q; radix 16 over q, twiddle
    // w_{16 R3}^{a2 s2}
    {
      const float2* pr = lds + cb * X + a0 * S1 + s2;
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = pr[q * R3];
    }
    idft16(x);
#pragma unroll
    for (int a2 = 1; a2 < 16; ++a2) x[a2] = cmul(x[a2], t2l[(a2 - 1) * R3]);
    // exchange 2 (inside the wave, in its own column region, which no
    // other wave reads): row d = a0 + 16 a2 at position s2, then rows
    // d = tb + Lp i at every position s
    {
      float2* pw = lds + cb * X + s2 * RS + a0;
#pragma unroll
      for (int a2 = 0; a2 < 16; ++a2) pw[16 * a2] = x[a2];
    }
    wave_lds_sync();
    {
      const float2* pr = lds + cb * X + tb;
#pragma unroll
      for (int s = 0; s < R3; ++s)
#pragma unroll
        for (int i = 0; i < 16 / R3; ++i) x[i * R3 + s] = pr[s * RS + Lp * i];
    }
    idft_groups<R3>(x);

    // post-pass of this wave's samples: register r holds j1 = tb +
    // Col::off(r) of column j2 = tile J + cb
    using K = Col<N1, J>;
    const unsigned j2 = tile * J + cb;
    auto jof = [&](int kk) {
      return j2 + (unsigned)N2 * (unsigned)K::out((int)tb, K::reg_by_order(kk));
    };
    float r2[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const float2 z = x[K::reg_by_order(kk)];
      r2[kk] = fmaf(z.x, z.x, z.y * z.y);
    }
    if (!a.full) {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const int j = (int)jof(kk);
        if (j < a.jlo32 || j >= a.jhi32) r2[kk] = -1.f;
      }
    }
    wave_post<16>(r2, jof, a, b, ((size_t)b * TILES + tile) * W::NW + wave, lane);
  };

  constexpr unsigned QS = Lp * N2 * (unsigned)sizeof(float2);
  const unsigned voff = p2_lane_off<N1, N2, C>(cc, t & ~1u) + (t & 1u) * QS;
  f4s vn[8];
  const int G = gridDim.x;
  int item = blockIdx.x;
  if (item < total) load_item_pairs<N1, N2, C, J>(vn, a, item, voff);
  for (; item < total; item += G) {
    float2 x[16];
    unpair_item(vn, x);
    if (item + G < total) load_item_pairs<N1, N2, C, J>(vn, a, item + G, voff);
    tile_body(x, item);
  }
}

// ---------------------------------------------------------------------------
// split-precision second pass: a radix-R3 stage on the vector units, then
// two radix-16 DFT-matrix stages on the matrix cores.  For a column of
// length L = 256 R3, with m = u + 256 p and n = b + R3 (v1 + 16 v0):
//   A[b][u]          = sum_p X[u + 256 p] w_R3^{b p}
//   B[b][u0][v1]     = sum_u1 w16^{v1 u1} w_L^{16 b u1} A[b][u0 + 16 u1]
//   Y[b + R3 v1 + 16 R3 v0] = sum_u0 w16^{v0 u0} w_L^{u0 (b + R3 v1)} B[b][u0][v1]
// The twiddle of the radix-R3 stage is split between the stage-B matrix
// (its u1 part, one matrix per b) and the twiddle before stage C (its u0
// part, merged with the four-step twiddle of the 256-point DFT).
// ---------------------------------------------------------------------------

// Operand fragments of the matrices for column length L: for mi < R3 the
// stage-B matrix M_mi[v][q] = w16^{v q} w_L^{16 mi q}, for mi = R3 the plain
// w16^{v q}.  Lane l holds output row v = l % 16 and inputs
// q = 4 (l / 16) + e / 2 (e < 8, real and imaginary parts interleaved along
// k) of the real rows [Re, -Im] and imaginary rows [Im, Re], split into high
// and low parts: out[(mi 4 + f) 64 + l], f = re_hi, re_lo, im_hi, im_lo
// (fragment-major, so the lanes of one read hit consecutive 16-byte words).
template <int PREC>
__global__ void k_mx_table(int L, const double2* __restrict__ tw64, uint4* __restrict__ out) {
  typedef typename MxT<PREC>::v8 V8;
  typedef typename MxT<PREC>::s S;
  const int mi = blockIdx.x, l = threadIdx.x;
  const int R3 = L / 256, v = l % 16, g = l / 16;
  V8 f[4];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int q = 4 * g + e / 2;
    int E = (L / 16) * v * q + (mi < R3 ? 16 * mi * q : 0);
    E %= L;
    const double2 w = tw64[E * (2048 / L)];
    const float re = (e & 1) ? (float)(-w.y) : (float)w.x;
    const float im = (e & 1) ? (float)w.x : (float)w.y;
    const S rh = (S)re, ih = (S)im;
    f[0][e] = rh;
    f[1][e] = (S)(re - (float)rh);
    f[2][e] = ih;
    f[3][e] = (S)(im - (float)ih);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) out[(mi * 4 + k) * 64 + l] = __builtin_bit_cast(uint4, f[k]);
}

template <int R>
__device__ __forceinline__ void idft_r(float2 (&x)[R]) {
  if constexpr (R == 2) {
    idft2(x[0], x[1]);
  } else if constexpr (R == 4) {
    idft4(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 8) {
    float2 t[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = x[i];
    idft8<0>(t);
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = t[i];
  }
}


constexpr int kXS = 18;  // row stride (complex) of the stage-C exchange

template <int L>
constexpr size_t p2mx_lds_bytes(int J) {
  return sizeof(float2) * L + sizeof(uint4) * (L / 256 + 1) * 256 +
         sizeof(float2) * 16 * kXS * (size_t)J;
}

// Persistent split-precision pass 2: wave w of a workgroup transforms
// column j2 = tile J + w; lane (u0 = l % 16, g = l / 16) loads
// X[u0 + 16 (4 g + e) + 256 p] (e < 4, p < R3) from the FP16 intermediate.
// MODE 0: post-pass (peaks and window keys); MODE 1: store the series.
template <int N1, int N2, int C, int J, int PREC, int MODE>
__global__ __launch_bounds__(J * 64, N1 <= 1024 ? 4 : 1) void k_p2mx(P2Args a) {
  constexpr int L = N1, R3 = L / 256, N = N1 * N2, TILES = N2 / J;
  typedef typename MxT<PREC>::v8 V8;
  extern __shared__ float2 lds[];
  // tws[(b 4 + e) 64 + l] = w_L^{u0 (b + R3 v1)} for lane l = u0 + 16 g,
  // v1 = 4 g + e (the twiddle before stage C): a lane reads its sixteen at
  // fixed offsets from one base address
  float2* tws = lds;
  const uint4* afr = reinterpret_cast<const uint4*>(lds + L);
  const unsigned tid = threadIdx.x, lane = tid & 63;
  const unsigned wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const unsigned u0 = lane & 15, g = lane >> 4;
  float2* xw = lds + L + (R3 + 1) * 256 * 2 + wave * 16 * kXS;
  {
    uint4* af = reinterpret_cast<uint4*>(lds + L);
    for (int k = tid; k < L; k += J * 64) {
      const unsigned l = k & 63, be = k >> 6, ub = l & 15, gb = l >> 4;
      const unsigned E = (ub * (be / 4 + R3 * (4 * gb + be % 4))) & (L - 1);
      tws[k] = a.tw[E * (2048 / L)];
    }
    for (int k = tid; k < (R3 + 1) * 256; k += J * 64) af[k] = a.mxa[k];
  }
  __syncthreads();
  const float2* twt = tws + lane;
  // byte offset of the lane's first input (k1 = u0 + 64 g) from the base of
  // its column; input (p, e) adds k1 += 16 e + 256 p, a constant offset
  const unsigned voff =
      ((u0 / C + (64 / C) * g) * N2 * C + u0 % C) * (unsigned)sizeof(unsigned);
  V8 wc[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) wc[f] = __builtin_bit_cast(V8, afr[(R3 * 4 + f) * 64 + lane]);
  const int total = a.nb * TILES;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int bt = item / TILES, tile = item % TILES;
    const unsigned j2 = tile * J + wave;
    float2 x[R3][4];
    {
      // column j2 of template bt: k1 = u0 + 16 (4 g + e) + 256 p lies at
      // ((k1 / C) N2 + j2) C + k1 % C, the lane's offset plus a constant
      const __amdgpu_buffer_rsrc_t r =
          buf_rsrc(reinterpret_cast<const unsigned*>(a.y) + (size_t)bt * N + (size_t)j2 * C,
                   (unsigned)(N - j2 * C) * (unsigned)sizeof(unsigned));
      unsigned raw[R3][4];
#pragma unroll
      for (int p = 0; p < R3; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          raw[p][e] = buf_ld(r, voff, ((16 / C) * e + (256 / C) * p) * N2 * C *
                                          (unsigned)sizeof(unsigned));
      if constexpr (PREC == kFP16 && R3 <= 4) {
        // the FP16 path: stages A and B on the matrix cores from the stored
        // words (exact FP16 operands, no conversion, no operand split)
        f16x8 A[R3][4];
#pragma unroll
        for (int b = 0; b < R3; ++b)
#pragma unroll
          for (int f = 0; f < 4; ++f) A[b][f] = __builtin_bit_cast(f16x8, afr[(b * 4 + f) * 64 + lane]);
        f32x4 yr[R3], yi[R3];
        mx_ab_f16<R3>(raw, A, yr, yi);
#pragma unroll
        for (int b = 0; b < R3; ++b)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            x[b][e] = cmul(make_float2(yr[b][e], yi[b][e]), twt[(b * 4 + e) * 64]);
      } else {
#pragma unroll
        for (int p = 0; p < R3; ++p)
#pragma unroll
          for (int e = 0; e < 4; ++e) x[p][e] = h2f(raw[p][e]);
      }
    }
    constexpr bool kFoldAB = PREC == kFP16 && R3 <= 4;
    // FP16 operand range: the radix-R3 stage and a radix-16 stage grow
    // magnitudes by at most 16 R3, so inputs within kF16Lim / (16 R3) keep
    // every operand of both matrix-core stages within the limit and the
    // per-instance check can be skipped for this tile (with stages A and B
    // done from the stored words, only stage C's operands are checked:
    // x then holds its inputs, which a radix-16 stage grows at most 16-fold)
    bool guard = false;
    if constexpr (kFoldAB) {
      float m = 0.f;
#pragma unroll
      for (int b = 0; b < R3; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) m = fmaxf(m, fmaxf(fabsf(x[b][e].x), fabsf(x[b][e].y)));
      guard = __any(!(m <= kF16Lim / 16.0f));
    } else if constexpr (PREC == kFP16) {
      float m = 0.f;
#pragma unroll
      for (int p = 0; p < R3; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) m = fmaxf(m, fmaxf(fabsf(x[p][e].x), fabsf(x[p][e].y)));
      guard = __any(!(m <= kF16Lim / (16.0f * R3)));
    }
    // stage A: radix-R3 over p
    if constexpr (R3 > 1 && !kFoldAB) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float2 t[R3];
#pragma unroll
        for (int p = 0; p < R3; ++p) t[p] = x[p][e];
        idft_r<R3>(t);
#pragma unroll
        for (int p = 0; p < R3; ++p) x[p][e] = t[p];
      }
    }
    // stage B with the folded twiddle, then w_L^{u0 (b + R3 v1)}
#pragma unroll
    for (int b = 0; b < (kFoldAB ? 0 : R3); ++b) {
      V8 A4[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) A4[f] = __builtin_bit_cast(V8, afr[(b * 4 + f) * 64 + lane]);
      float v[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[2 * e] = x[b][e].x;
        v[2 * e + 1] = x[b][e].y;
      }
      f32x4 yr, yi;
      mx_prod<PREC>(A4, v, yr, yi, guard);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[b][e] = cmul(make_float2(yr[e], yi[e]), twt[(b * 4 + e) * 64]);
    }
    // stage C per b through this wave's exchange rows: lane (u0, g) holds
    // v1 = 4 g + e; afterwards lane (v1 = l % 16, g) holds u0 = 4 g + e
#pragma unroll
    for (int b = 0; b < R3; ++b) {
#pragma unroll
      for (int e = 0; e < 4; ++e) xw[(4 * g + e) * kXS + u0] = x[b][e];
      wave_lds_sync();
      const float4* rp = reinterpret_cast<const float4*>(xw + u0 * kXS + 4 * g);
      const float4 r0 = rp[0], r1 = rp[1];
      wave_lds_sync();
      const float v[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
      f32x4 yr, yi;
      mx_prod<PREC>(wc, v, yr, yi, guard);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[b][e] = make_float2(yr[e], yi[e]);
    }
    // x[b][e] = z at n = b + R3 v1 + 16 R3 (4 g + e), v1 = u0
    if constexpr (MODE == 1) {
      float2* zt = a.z + (size_t)bt * N + j2;
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int b = 0; b < R3; ++b)
          zt[(size_t)N2 * (b + R3 * u0 + 16 * R3 * (4 * g + e))] = x[b][e];
    } else {
      // visited in increasing n = b + R3 v1 + 16 R3 (4 g + e)
      auto jof = [&](int i) {
        const int e = i / R3, b = i % R3;
        return j2 + (unsigned)N2 * (unsigned)(b + R3 * (int)u0 + 16 * R3 * (4 * (int)g + e));
      };
      float r2[4 * R3];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int b = 0; b < R3; ++b) r2[e * R3 + b] = fmaf(x[b][e].x, x[b][e].x, x[b][e].y * x[b][e].y);
      if (!a.full) {
#pragma unroll
        for (int i = 0; i < 4 * R3; ++i) {
          const int j = (int)jof(i);
          if (j < a.jlo32 || j >= a.jhi32) r2[i] = -1.f;
        }
      }
      // one peak partial per column (wave)
      wave_post<4 * R3>(r2, jof, a, bt, (size_t)bt * N2 + j2, lane);
    }
  }
}

// Per-batch finalisation: one workgroup per template reduces the pass-2
// partials to the peak, recomputes z at the peak and at every window
// trigger, and compacts the triggers.  k_place, launched after it on the
// same stream, then places the batch's triggers (or merges them) in order:
// the kernel boundary makes every workgroup's results visible to it, with
// no device-scope fence (each of which writes back a whole L2) inside
// either kernel.
// At most 128 registers up to n1 = 1024, so that the finalisers take less
// of the register file from the first pass they overlap; at 2048 the
// column's FP64 recompute needs more than 256, so one wave per SIMD.
template <int N1, int N2, int C>
__global__ __launch_bounds__(256, N1 <= 1024 ? 4 : 1) void k_fin(P2Args a) {
  extern __shared__ float2 lds[];
  finalize_template<N1, N2, C>(a, blockIdx.x, lds);
}

__global__ __launch_bounds__(256) void k_place(P2Args a) {
  extern __shared__ float2 lds[];
  place_batch(a, lds);
}

template <int N1, int N2, int C, int J>
__global__ __launch_bounds__(J * N1 / 16) void k_pass2_series(P2Args a) {
  constexpr int N = N1 * N2;
  constexpr int TILES = N2 / J;
  extern __shared__ float2 lds[];
  const unsigned tid = threadIdx.x;
  const unsigned cc = tid % J, t = tid / J;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int b = bid / TILES, tile = bid % TILES;
  const unsigned j2 = tile * J + cc;
  const float2* yb = a.y + (size_t)b * N;

  float2 x[16];
  load_pass2<N1, N2, C, J>(x, yb, j2, t);
  fft_col<N1, J>(x, lds, t, cc, a.tw);

  // non-temporal like the intermediate (a batch of series outlasts every
  // cache; measured: the two-polarization form 1 % faster)
  float2* zt = a.z + (size_t)b * N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j1 = Col<N1, J>::out(t, r);
    st_nt(&zt[j2 + N2 * j1], x[r]);
  }
}

__global__ void k_init_call(ci_trigger* mrec, int nwin, u64* run, int64_t* d_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwin) {
    ci_trigger e;
    e.tmpl = -1; e.index = -1; e.rho2 = -1.f; e.re = 0.f; e.im = 0.f; e.window = -1;
    mrec[i] = e;
  }
  if (i == 0) {
    run[0] = 0ull;
    d_count[0] = 0;
  }
}

// ---------------------------------------------------------------------------
// merge of two per-window trigger lists (chunks of one bank)
// ---------------------------------------------------------------------------

// Per-window records start empty.
__global__ void k_merge_clear(ci_trigger* __restrict__ dense, int64_t nwin) {
  const int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (w < nwin) {
    ci_trigger e;
    e.tmpl = -1; e.index = -1; e.rho2 = -1.f; e.re = 0.f; e.im = 0.f; e.window = -1;
    dense[w] = e;
  }
}

// One list into the per-window records: its entry replaces the window's
// record when that is empty or strictly smaller, so of two lists scattered
// in turn the first keeps the window on equal rho^2 (the earlier chunk's,
// smaller template).  Each list holds at most one entry per window, so no
// two lanes of one launch write the same record.
__global__ void k_merge_scatter(const ci_trigger* __restrict__ src, const int64_t* __restrict__ cnt,
                                int64_t cap, int64_t off, int64_t nwin,
                                ci_trigger* __restrict__ dense) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = cnt[0] < cap ? cnt[0] : cap;
  if (i >= n) return;
  ci_trigger e = src[i];
  if (e.tmpl < 0 || e.window < 0 || e.window >= nwin) return;
  e.tmpl += off;
  const ci_trigger cur = dense[e.window];
  if (cur.tmpl < 0 || e.rho2 > cur.rho2) dense[e.window] = e;
}

// Compaction of the records in window order (one workgroup).
__global__ __launch_bounds__(256) void k_merge_compact(const ci_trigger* __restrict__ dense,
                                                       int64_t nwin, ci_trigger* __restrict__ out,
                                                       int64_t cap, int64_t* __restrict__ d_count) {
  __shared__ int sh[256];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t per = (nwin + nt - 1) / nt;
  const int64_t w0 = tid * per, w1 = w0 + per < nwin ? w0 + per : nwin;
  int mine = 0;
  for (int64_t w = w0; w < w1; ++w) mine += dense[w].tmpl >= 0;
  int total = 0;
  int64_t pos = block_excl_scan(mine, sh, &total);
  for (int64_t w = w0; w < w1; ++w) {
    const ci_trigger e = dense[w];
    if (e.tmpl >= 0) {
      if (pos < cap) out[pos] = e;
      ++pos;
    }
  }
  if (tid == 0) d_count[0] = total;
}

hipError_t launch_merge(const ci_trigger* a, const int64_t* ca, int64_t cap_a, const ci_trigger* b,
                        const int64_t* cb, int64_t cap_b, int64_t off_b, int64_t nwin,
                        ci_trigger* dense, ci_trigger* out, int64_t cap, int64_t* d_count,
                        hipStream_t st) {
  // a list holds at most one entry per window: nwin bounds its grid
  if (cap_a > nwin) cap_a = nwin;
  if (cap_b > nwin) cap_b = nwin;
  const unsigned gw = (unsigned)((nwin + 255) / 256);
  hipLaunchKernelGGL(k_merge_clear, dim3(gw), dim3(256), 0, st, dense, nwin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (cap_a > 0) {
    hipLaunchKernelGGL(k_merge_scatter, dim3((unsigned)((cap_a + 255) / 256)), dim3(256), 0, st,
                       a, ca, cap_a, (int64_t)0, nwin, dense);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (cap_b > 0) {
    hipLaunchKernelGGL(k_merge_scatter, dim3((unsigned)((cap_b + 255) / 256)), dim3(256), 0, st,
                       b, cb, cap_b, off_b, nwin, dense);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_merge_compact, dim3(1), dim3(256), 0, st, dense, nwin, out, cap, d_count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// streaming bandwidth probes (the device's write, read and copy ceilings)
// ---------------------------------------------------------------------------

// Grid-stride loops over 16-byte elements, four in flight per lane, with
// the non-temporal hints the search's intermediate uses.
typedef float f4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_probe_write(f4v* __restrict__ p, int64_t n4, float v) {
  const int64_t g = (int64_t)gridDim.x * 256;
  const f4v w = {v, v, v, v};
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n4; i += 4 * g) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * g < n4) __builtin_nontemporal_store(w, &p[i + u * g]);
  }
}

__global__ __launch_bounds__(256) void k_probe_read(const f4v* __restrict__ p, int64_t n4,
                                                     float* __restrict__ sink) {
  const int64_t g = (int64_t)gridDim.x * 256;
  float acc = 0.f;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n4; i += 4 * g) {
    f4v v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f4v z = {0.f, 0.f, 0.f, 0.f};
      v[u] = i + u * g < n4 ? __builtin_nontemporal_load(&p[i + u * g]) : z;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  // never true for the probe's data (zeros): keeps the loads alive
  if (acc == 12345.f) sink[0] = acc;
}

__global__ __launch_bounds__(256) void k_probe_copy(const f4v* __restrict__ src,
                                                     f4v* __restrict__ dst, int64_t n4) {
  const int64_t g = (int64_t)gridDim.x * 256;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n4; i += 4 * g) {
    f4v v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * g < n4) v[u] = __builtin_nontemporal_load(&src[i + u * g]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * g < n4) __builtin_nontemporal_store(v[u], &dst[i + u * g]);
  }
}

hipError_t launch_probe(int kind, void* buf, int64_t bytes, int blocks, hipStream_t st) {
  const int64_t n4 = bytes / 16;
  f4v* p = static_cast<f4v*>(buf);
  if (kind == 0)
    hipLaunchKernelGGL(k_probe_write, dim3(blocks), dim3(256), 0, st, p, n4, 0.f);
  else if (kind == 1)
    hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(256), 0, st, p, n4,
                       reinterpret_cast<float*>(p));
  else
    hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, st, p, p + n4, n4);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// chi-squared veto at trigger samples
// ---------------------------------------------------------------------------

constexpr int kChiThreads = 512;
constexpr int kChiMaxBands = 64;

// Sum of a double2 over the workgroup (every thread gets the result).
__device__ __forceinline__ double2 block_sum_d2(double2 v, double2* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  for (int w = 0; w < kChiThreads / 64; ++w) {
    t.x += sh[w].x;
    t.y += sh[w].y;
  }
  return t;
}

// One workgroup per trigger: band edges by binary search of the FP64
// running sum of 4 df f^{-7/3} / S (the template's sigma^2 up to bin k),
// band-limited SNR z_l at the trigger's sample j with
//   Z_k exp(2 pi i j k / n) = scale w_k exp(2 pi i (Psi_k / 2 pi + j k / n)),
// the phase fraction formed in FP64 and the terms accumulated in FP64, and
// chi2 = p sum_l |z_l - z / p|^2 with z = sum_l z_l.
__global__ __launch_bounds__(kChiThreads) void k_chisq(const SegDev* __restrict__ sd,
                                                       const ci_tparams* __restrict__ prm,
                                                       int64_t ntmpl,
                                                       const float2* __restrict__ w,
                                                       const double* __restrict__ psum,
                                                       const ci_trigger* __restrict__ trig,
                                                       int bands, double* __restrict__ out) {
  __shared__ int s_edge[kChiMaxBands + 1];
  __shared__ double2 s_red[kChiThreads / 64];
  __shared__ double2 s_zl[kChiMaxBands];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const ci_trigger tr = trig[i];
  const int64_t n = sd->n;
  const bool valid_idx = tr.tmpl >= 0 && tr.tmpl < ntmpl && tr.index >= 0 && tr.index < n;
  ci_tparams P;
  if (valid_idx) P = prm[tr.tmpl];
  if (!valid_idx || P.k_high < P.k_low || (P.flags & CI_TMPL_EMPTY)) {
    if (tid == 0) out[i] = __builtin_nan("");
    return;
  }
  const int kl = P.k_low, kh = P.k_high;
  const double total = psum[kh];
  if (tid == 0) {
    s_edge[0] = kl;
    s_edge[bands] = kh + 1;
  }
  if (tid >= 1 && tid < bands) {
    // first k in [kl, kh] with psum[k] >= (tid / bands) total
    const double thr = total * (double)tid / (double)bands;
    int lo = kl, hi = kh;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      if (psum[mid] >= thr) hi = mid;
      else lo = mid + 1;
    }
    s_edge[tid] = lo;
  }
  __syncthreads();
  // n is a power of two: (j k) mod n is a mask
  const uint64_t j = (uint64_t)tr.index, nmask = (uint64_t)n - 1;
  const double inv_n = 1.0 / (double)n;
  for (int l = 0; l < bands; ++l) {
    double2 acc = make_double2(0.0, 0.0);
    for (int k = s_edge[l] + tid; k < s_edge[l + 1]; k += kChiThreads) {
      double f = (double)phase_frac(P, k) + (double)((j * (uint64_t)k) & nmask) * inv_n;
      f -= rint(f);
      const float fr = (float)f;
      const float2 e = make_float2(__builtin_amdgcn_cosf(fr) * P.scale,
                                   __builtin_amdgcn_sinf(fr) * P.scale);
      const float2 t = cmul(w[k], e);
      acc.x += (double)t.x;
      acc.y += (double)t.y;
    }
    const double2 zl = block_sum_d2(acc, s_red);
    if (tid == 0) s_zl[l] = zl;
  }
  __syncthreads();
  if (tid == 0) {
    double zr = 0.0, zi = 0.0;
    for (int l = 0; l < bands; ++l) {
      zr += s_zl[l].x;
      zi += s_zl[l].y;
    }
    const double pr = zr / bands, pi = zi / bands;
    double c = 0.0;
    for (int l = 0; l < bands; ++l) {
      const double dr = s_zl[l].x - pr, di = s_zl[l].y - pi;
      c += dr * dr + di * di;
    }
    out[i] = bands * c;
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

Plan plan_for(int log2n, int c, int j, int precision) {
  Plan p;
  p.log2n = log2n;
  switch (log2n) {
    case 16: p.n1 = 256; p.n2 = 256; break;
    case 17: p.n1 = 512; p.n2 = 256; break;
    case 18: p.n1 = 512; p.n2 = 512; break;
    case 19: p.n1 = 1024; p.n2 = 512; break;
    case 20: p.n1 = 1024; p.n2 = 1024; break;
    case 21:
      // FP32: 1024-point second-pass columns (wave-owned, ~5.0 TB/s against
      // ~3.5 for 2048-point ones), 2048-point first-pass columns; the split
      // paths keep 2048 x 1024, where their first pass is faster
      p.n1 = precision == CI_FP32 ? 1024 : 2048;
      p.n2 = precision == CI_FP32 ? 2048 : 1024;
      break;
    default: p.n1 = p.n2 = 0;
  }
  p.c = (c == 4 || c == 8) ? c : 4;
  p.j = (j == 4 || j == 8) ? j : 4;
  return p;
}

hipError_t launch_segment_powers(Seg* s, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_powers, dim3(1024), dim3(256), 0, st, s->dev, s->fpw);
  return hipGetLastError();
}

hipError_t launch_segment(Seg* s, const void* d_xtilde, const double* d_psd, hipStream_t st) {
  const int nblk = (int)(s->host.half / kSegBlock);
  hipLaunchKernelGGL(k_seg_terms, dim3(nblk), dim3(kSegThreads), 0, st, s->dev, d_psd, s->fpw,
                     s->psum, s->bsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, st, s->dev, s->bsum, nblk);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_final, dim3(nblk), dim3(kSegThreads), 0, st, s->dev,
                     reinterpret_cast<const float2*>(d_xtilde), d_psd, s->psum, s->bsum, s->w,
                     s->w0, s->isp, s->fpw);
  return hipGetLastError();
}

hipError_t launch_params(const Seg* s, ci_tparams* d_params, int64_t n, void* d_htilde,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_params, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s->dev,
                     s->psum, d_params, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || d_htilde == nullptr) return e;
  const int64_t m = s->host.half + 1;
  int bx = (int)((m + 255) / 256);
  if (bx > 1024) bx = 1024;
  for (int64_t t0 = 0; t0 < n; t0 += 65535) {
    const int64_t cnt = (n - t0 < 65535) ? n - t0 : 65535;
    hipLaunchKernelGGL(k_htilde, dim3(bx, (unsigned)cnt), dim3(256), 0, st, s->dev,
                       d_params + t0, reinterpret_cast<float2*>(d_htilde) + t0 * m);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_chisq(const Seg* s, const ci_tparams* d_params, int64_t ntmpl,
                        const ci_trigger* d_trig, int64_t ntrig, int bands, double* d_out,
                        hipStream_t st) {
  for (int64_t t0 = 0; t0 < ntrig; t0 += 65535 * 64) {
    const int64_t cnt = (ntrig - t0 < 65535 * 64) ? ntrig - t0 : 65535 * 64;
    hipLaunchKernelGGL(k_chisq, dim3((unsigned)cnt), dim3(kChiThreads), 0, st, s->dev, d_params,
                       ntmpl, s->w, s->psum, d_trig + t0, bands, d_out + t0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_init_call(const TrigWork& tw, int nwin, int64_t* d_count, hipStream_t st) {
  const int blocks = (nwin + 255) / 256 + 1;
  hipLaunchKernelGGL(k_init_call, dim3(blocks), dim3(256), 0, st, tw.mrec, nwin, tw.run,
                     d_count);
  return hipGetLastError();
}

namespace {

// finaliser LDS: 2 doubles per lane (256 lanes) or one int per template of
// the batch (<= 4096)
constexpr size_t kFinLds = 16384;

template <typename K>
hipError_t set_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

P1Args make_p1(const BatchArgs& a, bool zero_trig) {
  P1Args p;
  p.prm = a.params;
  p.w = a.seg->w;
  p.tw = a.seg->tw2048;
  p.twa = a.seg->twa;
  p.twb = a.seg->twb;
  p.tw64 = a.seg->tw64;
  p.y = a.y;
  p.nb = a.nb;
  p.uv = a.uv;
  p.tdp = a.td;
  p.w0 = a.seg->w0;
  p.sig = a.sig;
  p.sd = a.seg->dev;
  if (zero_trig) {
    const int s = a.slot;
    p.wkeys = a.tw.wkeys + (size_t)s * a.bmax * a.nwin;
    p.nzero_w = (int64_t)a.nb * a.nwin;
    p.mkey = a.tw.mkey + (size_t)s * a.nwin;
    p.nwin = a.nwin;
  } else {
    p.wkeys = nullptr;
    p.nzero_w = 0;
    p.mkey = nullptr;
    p.nwin = 0;
  }
  return p;
}

// The wave-owned-column second pass applies to FP32 searches at n1 = 512
// or 1024.
bool uses_p2_wave(const BatchArgs& a) {
  return a.p2_wave && a.precision == CI_FP32 && !a.d_z && (a.plan.n1 == 512 || a.plan.n1 == 1024);
}

P2Args make_p2(const BatchArgs& a) {
  P2Args p;
  const int s = a.slot;
  if (a.td) {
    p.flagp = reinterpret_cast<const char*>(&a.td->flags);
    p.flag_stride = (int)sizeof(ci_tdparams);
  } else if (a.params) {
    p.flagp = reinterpret_cast<const char*>(&a.params->flags);
    p.flag_stride = (int)sizeof(ci_tparams);
  } else {
    // plain transforms (series mode without templates): no finaliser
    p.flagp = nullptr;
    p.flag_stride = 0;
  }
  p.tw = a.seg->tw2048;
  p.tw64 = a.seg->tw64;
  p.y = a.y;
  p.t0 = a.t0;
  p.nb = a.nb;
  // peak partials per template: one per second-pass workgroup, or one per
  // wave with wave-owned columns (one per column on the split-precision
  // paths); slot sets are sized for n2 per template
  p.ntile2 = uses_p2_wave(a) ? a.plan.n2 * (a.plan.n1 / 16) / 64
             : (a.precision != CI_FP32 && !a.d_z) ? a.plan.n2
                                                   : a.plan.n2 / a.plan.j;
  p.ppart = a.tw.ppart ? a.tw.ppart + (size_t)s * a.bmax * a.plan.n2 : nullptr;
  p.wkeys = a.tw.wkeys ? a.tw.wkeys + (size_t)s * a.bmax * a.nwin : nullptr;
  p.mkey = a.tw.mkey ? a.tw.mkey + (size_t)s * a.nwin : nullptr;
  p.cnt = a.tw.cnt ? a.tw.cnt + (size_t)s * a.bmax : nullptr;
  p.sidx = a.tw.sidx ? a.tw.sidx + (size_t)s * a.bmax * a.nwin : nullptr;
  p.stage = a.tw.stage ? a.tw.stage + (size_t)s * a.bmax * a.nwin : nullptr;
  p.mrec = a.tw.mrec;
  p.run = a.tw.run;
  p.nwin = a.nwin;
  p.window = a.window;
  p.j_lo = a.j_lo;
  p.j_hi = a.j_hi;
  p.jlo32 = (int)a.j_lo;
  p.jhi32 = (int)a.j_hi;
  p.full = (a.j_lo == 0 && a.j_hi == a.seg->host.n) ? 1 : 0;
  p.win32 = (unsigned int)(a.window > 0 ? a.window : 1);
  p.thr2 = a.thr2;
  p.d_peaks = a.d_peaks;
  p.d_trig = a.d_trig;
  p.cap = a.cap;
  p.d_count = a.d_count;
  p.merge = a.merge;
  p.last_batch = a.last_batch;
  p.z = a.d_z;
  p.half_y = a.precision != CI_FP32 ? 1 : 0;
  p.mxa = a.precision == CI_SPLIT_BF16   ? a.seg->mxa2[0]
          : a.precision == CI_SPLIT_FP16 ? a.seg->mxa2[1]
                                         : nullptr;
  return p;
}

// Launch on st; with the batch's timing events set, the launch itself
// records them when it starts and ends (no separate event packets).
template <typename K, typename Arg>
hipError_t launch_timed(K kern, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                        const BatchArgs& a, const Arg& arg) {
  if (a.ev0)
    hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)lds, st, a.ev0, a.ev1, 0u, arg);
  else
    hipLaunchKernelGGL(kern, grid, block, lds, st, arg);
  return hipGetLastError();
}

// Whether a kernel's dynamic plus static LDS fits one workgroup's limit.
template <typename K>
hipError_t lds_fits(K kern, size_t dyn) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern));
  if (e != hipSuccess) return e;
  int dev = 0, lim = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lim, hipDeviceAttributeSharedMemPerBlockOptin, dev);
  if (e != hipSuccess) return e;
  return dyn + fa.sharedSizeBytes <= (size_t)lim ? hipSuccess : hipErrorInvalidConfiguration;
}

template <int N1, int N2, int C, int J>
struct Inst {
  // every kernel a search (trigger or series mode) launches fits
  static hipError_t fits(int precision) {
    // per instantiation and precision: 0 unknown, else the cached answer
    static hipError_t known[3] = {hipSuccess, hipSuccess, hipSuccess};
    static bool have[3] = {false, false, false};
    if (precision < 0 || precision > 2) return hipErrorInvalidValue;
    if (have[precision]) return known[precision];
    hipError_t e;
    if (precision == CI_FP32) {
      e = lds_fits(k_pass1<N1, N2, C, false>, (size_t)(Col<N2, C>::LDS_ELEMS + N2) * sizeof(float2));
      if (e == hipSuccess)
        e = lds_fits(k_pass2_trig<N1, N2, C, J>,
                     (size_t)(Col<N1, J>::LDS_ELEMS + N1) * sizeof(float2));
      if (e == hipSuccess)
        e = lds_fits(k_pass2_series<N1, N2, C, J>, (size_t)Col<N1, J>::LDS_ELEMS * sizeof(float2));
      if constexpr (N1 == 512 || N1 == 1024)
        if (e == hipSuccess) e = lds_fits(k_pass2w<N1, N2, C, J>, WaveCol<N1, J>::lds_bytes());
    } else if (precision == CI_SPLIT_BF16) {
      e = lds_fits(k_pass1<N1, N2, C, true>, (size_t)(Col<N2, C>::LDS_ELEMS + N2) * sizeof(float2));
      if (e == hipSuccess) e = lds_fits(k_p2mx<N1, N2, C, J, kBF16, 0>, p2mx_lds_bytes<N1>(J));
      if (e == hipSuccess) e = lds_fits(k_p2mx<N1, N2, C, J, kBF16, 1>, p2mx_lds_bytes<N1>(J));
    } else {
      e = lds_fits(k_pass1<N1, N2, C, true>, (size_t)(Col<N2, C>::LDS_ELEMS + N2) * sizeof(float2));
      if (e == hipSuccess) e = lds_fits(k_p2mx<N1, N2, C, J, kFP16, 0>, p2mx_lds_bytes<N1>(J));
      if (e == hipSuccess) e = lds_fits(k_p2mx<N1, N2, C, J, kFP16, 1>, p2mx_lds_bytes<N1>(J));
    }
    if (e == hipSuccess) e = lds_fits(k_fin<N1, N2, C>, kFinLds);
    if (e == hipSuccess || e == hipErrorInvalidConfiguration) {
      known[precision] = e;
      have[precision] = true;
    }
    return e;
  }
  template <bool H>
  static hipError_t p1(const BatchArgs& a, bool zero, hipStream_t st) {
    const size_t lds = (size_t)(Col<N2, C>::LDS_ELEMS + N2) * sizeof(float2);
    auto kern = k_pass1<N1, N2, C, H>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    return launch_timed(kern, dim3((unsigned)(a.nb * (N1 / C))), dim3(C * N2 / 16), lds, st, a,
                        make_p1(a, zero));
  }
  template <int MODE>
  static hipError_t p1mem(const BatchArgs& a, bool zero, hipStream_t st) {
    const size_t lds = (size_t)(Col<N2, C>::LDS_ELEMS + N2) * sizeof(float2);
    auto kern = k_pass1_mem<N1, N2, C, MODE>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    return launch_timed(kern, dim3((unsigned)(a.nb * (N1 / C))), dim3(C * N2 / 16), lds, st, a,
                        make_p1(a, zero));
  }
  static hipError_t p2t(const BatchArgs& a, hipStream_t st) {
    const size_t lds = (size_t)(Col<N1, J>::LDS_ELEMS + N1) * sizeof(float2);
    auto kern = k_pass2_trig<N1, N2, C, J>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    // workgroups that fit at once, per CU, and the CU count (per instantiation)
    static int per_cu = 0, cus = 0;
    if (per_cu == 0) {
      int dev = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, J * N1 / 16, lds);
      if (e == hipSuccess) e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      if (per_cu < 1) per_cu = 1;
    }
    const int wpc = (a.p2_per_cu > 0 && a.p2_per_cu < per_cu) ? a.p2_per_cu : per_cu;
    const long long items = (long long)a.nb * (N2 / J);
    long long grid = (long long)wpc * cus;
    if (grid > items) grid = items;
    if (grid < 1) grid = 1;
    return launch_timed(kern, dim3((unsigned)grid), dim3(J * N1 / 16), lds, st, a, make_p2(a));
  }
  static hipError_t p2w(const BatchArgs& a, hipStream_t st) {
    if constexpr (N1 == 512 || N1 == 1024) {
      using W = WaveCol<N1, J>;
      const size_t lds = W::lds_bytes();
      auto kern = k_pass2w<N1, N2, C, J>;
      hipError_t e = set_lds(kern, lds);
      if (e != hipSuccess) return e;
      static int per_cu = 0, cus = 0;
      if (per_cu == 0) {
        int dev = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, J * N1 / 16, lds);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
      }
      const int wpc = (a.p2_per_cu > 0 && a.p2_per_cu < per_cu) ? a.p2_per_cu : per_cu;
      const long long items = (long long)a.nb * (N2 / J);
      long long grid = (long long)wpc * cus;
      if (grid > items) grid = items;
      if (grid < 1) grid = 1;
      return launch_timed(kern, dim3((unsigned)grid), dim3(J * N1 / 16), lds, st, a, make_p2(a));
    } else {
      return p2t(a, st);
    }
  }
  template <int PREC, int MODE>
  static hipError_t p2mx(const BatchArgs& a, hipStream_t st) {
    const size_t lds = p2mx_lds_bytes<N1>(J);
    auto kern = k_p2mx<N1, N2, C, J, PREC, MODE>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    static int per_cu = 0, cus = 0;
    if (per_cu == 0) {
      int dev = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, J * 64, lds);
      if (e == hipSuccess) e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      if (per_cu < 1) per_cu = 1;
    }
    const int wpc = (a.p2_per_cu > 0 && a.p2_per_cu < per_cu) ? a.p2_per_cu : per_cu;
    const long long items = (long long)a.nb * (N2 / J);
    long long grid = (long long)wpc * cus;
    if (grid > items) grid = items;
    if (grid < 1) grid = 1;
    return launch_timed(kern, dim3((unsigned)grid), dim3(J * 64), lds, st, a, make_p2(a));
  }
  static hipError_t fin(const BatchArgs& a, hipStream_t st) {
    const P2Args p = make_p2(a);
    hipLaunchKernelGGL((k_fin<N1, N2, C>), dim3((unsigned)a.nb), dim3(256), kFinLds, st, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_place, dim3(1), dim3(256), kFinLds, st, p);
    return hipGetLastError();
  }
  static hipError_t p2s(const BatchArgs& a, hipStream_t st) {
    const size_t lds = (size_t)Col<N1, J>::LDS_ELEMS * sizeof(float2);
    auto kern = k_pass2_series<N1, N2, C, J>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    return launch_timed(kern, dim3((unsigned)(a.nb * (N2 / J))), dim3(J * N1 / 16), lds, st, a,
                        make_p2(a));
  }
};

template <int C, int J, typename F>
hipError_t dispatch_n(const Plan& p, F f) {
  switch (p.log2n) {
    case 16: return f(Inst<256, 256, C, J>());
    case 17: return f(Inst<512, 256, C, J>());
    case 18: return f(Inst<512, 512, C, J>());
    case 19: return f(Inst<1024, 512, C, J>());
    case 20: return f(Inst<1024, 1024, C, J>());
    case 21:
      return p.n1 == 1024 ? f(Inst<1024, 2048, C, J>()) : f(Inst<2048, 1024, C, J>());
    default: return hipErrorInvalidValue;
  }
}

// Tile shapes: C k1-columns per pass-1 workgroup, J j2-columns per pass-2
// workgroup (4 or 8 each).
template <typename F>
hipError_t dispatch(const Plan& p, F f) {
  if (p.c == 4 && p.j == 4) return dispatch_n<4, 4>(p, f);
  if (p.c == 4 && p.j == 8) return dispatch_n<4, 8>(p, f);
  if (p.c == 8 && p.j == 4) return dispatch_n<8, 4>(p, f);
  if (p.c == 8 && p.j == 8) return dispatch_n<8, 8>(p, f);
  return hipErrorInvalidValue;
}

}  // namespace

// ---------------------------------------------------------------------------
// continuous stream: segment spectrum and PSD estimate
// ---------------------------------------------------------------------------

// Segment samples from the device ring (capacity rmask + 1, a power of two)
// as two complex inputs: x_j and w_j x_j, w_j = sin^2(pi j / n).
__global__ __launch_bounds__(256) void k_stream_gather(const float* __restrict__ ring,
                                                       int64_t rmask, int64_t start, int64_t n,
                                                       float2* __restrict__ uv) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const float x = ring[(start + j) & rmask];
  // sin^2(pi j/n) = (1 - cos(2 pi j/n)) / 2, the cosine in revolutions
  const float w = 0.5f * (1.f - __builtin_amdgcn_cosf((float)j / (float)n));
  uv[j] = make_float2(x, 0.f);
  uv[n + j] = make_float2(w * x, 0.f);
}

// From V = IDFT of the two inputs (real inputs, so the forward DFT is the
// conjugate): x~_k = dt conj(V0_k) and the periodogram
// P_k = 2 |dt V1_k|^2 / (T 3/8) in FP64, k = 0..n/2.
__global__ __launch_bounds__(256) void k_stream_spec(const float2* __restrict__ V, int64_t n,
                                                     double dt, float2* __restrict__ xt,
                                                     double* __restrict__ pg) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k > n / 2) return;
  const float2 a = V[k], b = V[n + k];
  xt[k] = make_float2((float)(dt * a.x), (float)(-dt * a.y));
  const double T = dt * (double)n;
  pg[k] = 2.0 * dt * dt * ((double)b.x * b.x + (double)b.y * b.y) / (T * 0.375);
}

// PSD estimate: the mean of the periodogram over the in-band bins
// [k - h, k + h] intersected with [kl, kh]; 0 outside [kl, kh].
__global__ __launch_bounds__(256) void k_stream_psd(const double* __restrict__ pg, int64_t kl,
                                                    int64_t kh, int h, int64_t half,
                                                    double* __restrict__ psd) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k > half) return;
  double v = 0.0;
  if (k >= kl && k <= kh) {
    const int64_t a = k - h > kl ? k - h : kl, b = k + h < kh ? k + h : kh;
    double s = 0.0;
    for (int64_t i = a; i <= b; ++i) s += pg[i];
    v = s / (double)(b - a + 1);
  }
  psd[k] = v;
}

// Welch's average over time: the segment's own estimate (in psd) goes to
// ring slot `cur`; psd becomes the mean of the last `cnt` slots, oldest
// first.
__global__ __launch_bounds__(256) void k_stream_avg(double* __restrict__ ring, int K, int cur,
                                                    int cnt, int64_t m, double* __restrict__ psd) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= m) return;
  ring[(size_t)cur * m + k] = psd[k];
  double s = 0.0;
  for (int i = 0; i < cnt; ++i) s += ring[(size_t)((cur - cnt + 1 + i + K) % K) * m + k];
  psd[k] = s / (double)cnt;
}

hipError_t launch_stream_avg(double* ring, int K, int cur, int cnt, int64_t m, double* psd,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_stream_avg, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, ring, K,
                     cur, cnt, m, psd);
  return hipGetLastError();
}

hipError_t launch_stream_spectra(const Seg* seg, const float* ring, int64_t rmask, int64_t start,
                                 float2* uv, float2* y, float2* xt, double* pg, double* psd,
                                 int h, hipStream_t st) {
  const SegDev& hd = seg->host;
  const int64_t n = hd.n;
  hipLaunchKernelGGL(k_stream_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ring,
                     rmask, start, n, uv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchArgs a = {};
  a.seg = seg;
  a.plan = seg->plan;
  a.nb = 2;
  a.bmax = 2;
  a.precision = CI_FP32;
  a.uv = uv;
  a.y = y;
  a.d_z = uv;
  e = dispatch(a.plan, [&](auto inst) {
    typedef decltype(inst) I;
    hipError_t r = I::template p1mem<0>(a, false, st);
    return r == hipSuccess ? I::p2s(a, st) : r;
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stream_spec, dim3((unsigned)((hd.half + 1 + 255) / 256)), dim3(256), 0, st,
                     uv, n, 1.0 / hd.fs, xt, pg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stream_psd, dim3((unsigned)((hd.half + 1 + 255) / 256)), dim3(256), 0, st,
                     pg, (int64_t)hd.k_low, hd.half - 1, h, hd.half, psd);
  return hipGetLastError();
}

hipError_t launch_td_gen(const BatchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_td_gen, dim3((unsigned)(a.seg->host.n / 256), (unsigned)a.nb), dim3(256),
                     0, st, a.seg->dev, a.td, a.uv);
  return hipGetLastError();
}

hipError_t launch_td_prep(const BatchArgs& a, hipStream_t st) {
  // V = IDFT(u), u generated inside the first pass, through the
  // intermediate into a.uv
  BatchArgs c = a;
  c.d_z = a.uv;
  hipError_t e = dispatch(c.plan, [&](auto inst) {
    typedef decltype(inst) I;
    hipError_t r = I::template p1mem<2>(c, false, st);
    return r == hipSuccess ? I::p2s(c, st) : r;
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_td_sigma, dim3(kTdChunks, (unsigned)a.nb), dim3(256), 0, st, a.seg->dev,
                     a.td, a.uv, a.seg->isp, a.sig);
  return hipGetLastError();
}

hipError_t launch_td_export(const BatchArgs& a, void* d_hf, double* d_sigma2, hipStream_t st) {
  const int64_t m = a.seg->host.half + 1;
  hipLaunchKernelGGL(k_td_export, dim3((unsigned)((m + 255) / 256), (unsigned)a.nb), dim3(256), 0,
                     st, a.seg->dev, a.uv, a.sig, reinterpret_cast<float2*>(d_hf), d_sigma2);
  return hipGetLastError();
}

hipError_t launch_pass1(const BatchArgs& a, bool zero_trig, hipStream_t st) {
  if (a.td)
    return dispatch(a.plan, [&](auto inst) {
      return decltype(inst)::template p1mem<1>(a, zero_trig, st);
    });
  return dispatch(a.plan, [&](auto inst) {
    typedef decltype(inst) I;
    // the split-precision paths keep the first pass on the vector units and
    // store its output as FP16 pairs
    if (a.precision != CI_FP32) return I::template p1<true>(a, zero_trig, st);
    return I::template p1<false>(a, zero_trig, st);
  });
}
hipError_t launch_pass2_trig(const BatchArgs& a, hipStream_t st) {
  return dispatch(a.plan, [&](auto inst) {
    typedef decltype(inst) I;
    if (a.precision == CI_SPLIT_BF16) return I::template p2mx<kBF16, 0>(a, st);
    if (a.precision == CI_SPLIT_FP16) return I::template p2mx<kFP16, 0>(a, st);
    if (uses_p2_wave(a)) return I::p2w(a, st);
    return I::p2t(a, st);
  });
}
hipError_t launch_mx_tables(Seg* s, hipStream_t st) {
  const int L = s->plan.n1;
  hipLaunchKernelGGL(k_mx_table<kBF16>, dim3(L / 256 + 1), dim3(64), 0, st, L, s->tw64, s->mxa2[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mx_table<kFP16>, dim3(L / 256 + 1), dim3(64), 0, st, L, s->tw64, s->mxa2[1]);
  return hipGetLastError();
}

hipError_t plan_fits(const Plan& p, int precision) {
  return dispatch(p, [&](auto inst) { return decltype(inst)::fits(precision); });
}
hipError_t launch_fin(const BatchArgs& a, hipStream_t st) {
  return dispatch(a.plan, [&](auto inst) { return decltype(inst)::fin(a, st); });
}
hipError_t launch_pass2_series(const BatchArgs& a, hipStream_t st) {
  return dispatch(a.plan, [&](auto inst) {
    typedef decltype(inst) I;
    if (a.precision == CI_SPLIT_BF16) return I::template p2mx<kBF16, 1>(a, st);
    if (a.precision == CI_SPLIT_FP16) return I::template p2mx<kFP16, 1>(a, st);
    return I::p2s(a, st);
  });
}

}  // namespace ci
