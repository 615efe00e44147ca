// mfma_device.h -- radix-16 DFT-matrix products on the gfx950 matrix cores.
//
// A radix-16 step Y_a = sum_q M_aq X_q over 16 independent instances is a
// real product of a 32 x 32 matrix and a 32 x 16 block, one 16x16x32 MFMA
// per output half, with the real and imaginary parts of the inputs
// interleaved along k (k = 2 q + part):
//   real outputs:      row a = [Re M_a0, -Im M_a0, Re M_a1, -Im M_a1, ...]
//   imaginary outputs: row a = [Im M_a0,  Re M_a0, Im M_a1,  Re M_a1, ...]
// Operands are split into a high and a low part in the 16-bit type
// (x = x_hi + x_lo, M = M_hi + M_lo) and three products
//   M_hi x_hi + M_hi x_lo + M_lo x_hi
// accumulate in FP32, which keeps ~2^-16 (BF16) or ~2^-21 (FP16) relative
// error per stage.  FP16 inputs are pre-scaled by 2^6 to stay clear of its
// subnormal range and the outputs scaled back exactly.
//
// Operand layouts of v_mfma_f32_16x16x32_{bf16,f16} (lane l, g = l / 16):
//   A[i][k]: i = l % 16, k = 8 g + e (e < 8)
//   B[k][j]: j = l % 16, k = 8 g + e
//   D[i][j]: j = l % 16, i = 4 g + e (e < 4)
// so lane l supplies complex inputs q = 4 g .. 4 g + 3 of instance l % 16
// as (re, im, re, im, ...) and receives outputs a = 4 g .. 4 g + 3 of that
// instance: the same four-per-lane shape on both sides.
#pragma once

#include <hip/hip_runtime.h>

namespace ci {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// precision tags (match CI_SPLIT_BF16 / CI_SPLIT_FP16)
constexpr int kBF16 = 1;
constexpr int kFP16 = 2;

template <int PREC>
struct MxT;
template <>
struct MxT<kBF16> {
  typedef bf16x8 v8;
  typedef __bf16 s;
  static constexpr float kPre = 1.0f;
  __device__ static __forceinline__ f32x4 mma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MxT<kFP16> {
  typedef f16x8 v8;
  typedef _Float16 s;
  static constexpr float kPre = 64.0f;
  __device__ static __forceinline__ f32x4 mma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Split 8 FP32 values into high and low 16-bit parts.
template <int PREC>
__device__ __forceinline__ void split8(const float (&v)[8], typename MxT<PREC>::v8& hi,
                                       typename MxT<PREC>::v8& lo) {
  typedef typename MxT<PREC>::s S;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x = v[e] * MxT<PREC>::kPre;
    const S h = (S)x;
    hi[e] = h;
    lo[e] = (S)(x - (float)h);
  }
}

// Split 8 FP32 values into the two 16-bit operands of a product.  BF16:
// the high part is the value truncated to BF16 (exact in FP32, so the low
// part x - hi is exact before its own rounding).  FP16: after the 2^6
// pre-scale, the high parts are rounded to nearest two at a time, and each
// low part x - hi comes from one mixed-precision FMA that reads the high
// part as FP16 and writes its FP16 result into its half of the packed word.
template <int PREC>
__device__ __forceinline__ void split8t(const float (&v)[8], typename MxT<PREC>::v8& hi,
                                        typename MxT<PREC>::v8& lo,
                                        float pre = MxT<PREC>::kPre) {
  if constexpr (PREC == kBF16) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const unsigned u = __builtin_bit_cast(unsigned, v[e]) & 0xffff0000u;
      hi[e] = __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
      lo[e] = (__bf16)(v[e] - __builtin_bit_cast(float, u));
    }
  } else {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    unsigned hw[4], lw[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float a = v[2 * i] * pre, b = v[2 * i + 1] * pre;
      h2 h;
      h.x = (_Float16)a;
      h.y = (_Float16)b;
      const unsigned hp = __builtin_bit_cast(unsigned, h);
      unsigned lp = 0u;
      asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "+v"(lp) : "v"(hp), "v"(a));
      asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
          : "+v"(lp) : "v"(hp), "v"(b));
      hw[i] = hp;
      lw[i] = lp;
    }
    hi = __builtin_bit_cast(typename MxT<PREC>::v8, make_uint4(hw[0], hw[1], hw[2], hw[3]));
    lo = __builtin_bit_cast(typename MxT<PREC>::v8, make_uint4(lw[0], lw[1], lw[2], lw[3]));
  }
}

// One DFT-matrix product on 16 instances with the operand layout that
// interleaves real and imaginary parts along k: the lane (j = l % 16,
// g = l / 16) supplies complex inputs q = 4 g .. 4 g + 3 of instance j as
// v = (re, im, re, im, ...), and A holds that lane's fragments of the
// matrix rows [Re, -Im] (real outputs) and [Im, Re] (imaginary outputs),
// high and low parts: A[0] re_hi, A[1] re_lo, A[2] im_hi, A[3] im_lo.
// Returns outputs v = 4 g .. 4 g + 3 of instance j.
//
// FP16 range: the 2^6 pre-scale keeps FP16 operands finite while an
// instance's inputs stay below 2^9 in magnitude.  When any input of a wave
// exceeds that (a loud signal or glitch), each instance whose largest input
// does gets its own power-of-two scale 2^(14 - floor(log2 max)) instead,
// which puts its largest operand in [2^14, 2^15); its outputs are scaled
// back exactly.  Instances below the limit keep the 2^6 pre-scale, so their
// results are unchanged bit for bit, and the scale depends only on the
// instance's own inputs (not on the launch configuration).
constexpr float kF16Lim = 512.0f;

// guard: false when the caller has shown that no input of this wave can
// exceed the limit (the per-instance check is then skipped).
template <int PREC>
__device__ __forceinline__ void mx_prod(const typename MxT<PREC>::v8 (&A)[4], const float (&v)[8],
                                        f32x4& yr, f32x4& yi, bool guard = true) {
  typedef MxT<PREC> M;
  float pre = M::kPre;
  if constexpr (PREC == kFP16) {
    if (!guard) goto split;
    float m = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) m = fmaxf(m, fabsf(v[e]));
    if (__any(!(m <= kF16Lim))) {
      // the instance's four lanes (l, l ^ 16, l ^ 32, l ^ 48) agree on it
      m = fmaxf(m, __shfl_xor(m, 16, 64));
      m = fmaxf(m, __shfl_xor(m, 32, 64));
      // m = f 2^e with f in [1/2, 1): 2^(15 - e) m lies in [2^14, 2^15)
      if (!(m <= kF16Lim)) pre = __builtin_amdgcn_ldexpf(1.0f, 15 - __builtin_amdgcn_frexp_expf(m));
    }
  }
split:
  typename M::v8 bh, bl;
  split8t<PREC>(v, bh, bl, pre);
  f32x4 z = {0.f, 0.f, 0.f, 0.f};
  yr = M::mma(A[0], bh, z);
  yi = M::mma(A[2], bh, z);
  yr = M::mma(A[0], bl, yr);
  yi = M::mma(A[2], bl, yi);
  yr = M::mma(A[1], bh, yr);
  yi = M::mma(A[3], bh, yi);
  if constexpr (M::kPre != 1.0f) {
    const float inv = 1.0f / pre;  // a power of two: exact
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      yr[e] *= inv;
      yi[e] *= inv;
    }
  }
}

// Stages A and B of a column of length 256 R3 (R3 <= 4) from exact FP16
// inputs.  Lane (u0, g) supplies raw[p][e] = X[u0 + 16 (4 g + e) + 256 p]
// as packed (re, im) FP16 words, which are the B operand as stored.  The
// radix-R3 factors w_R3^{b p} are 1, i, -1 or -i, so with (Re, Im) = the
// real- and imaginary-output products of stage B's matrix M_b with X_p,
//   sum_p w^{b p} (M_b X_p)  takes  (+Re, +Im), (-Im, +Re), (-Re, -Im) or
//   (+Im, -Re)  per term,
// accumulated into positive and negative FP32 accumulators (two products
// per matrix part: M = M_hi + M_lo; the data need no split) and differenced
// at the end: yr[b] + i yi[b] = M_b sum_p w^{b p} X_p for outputs
// v1 = 4 g .. 4 g + 3 of instance u0.  A[b] holds the fragments of M_b as
// mx_prod expects them (re_hi, re_lo, im_hi, im_lo).
template <int R3>
__device__ __forceinline__ void mx_ab_f16(const unsigned (&raw)[R3][4],
                                          const f16x8 (&A)[R3][4], f32x4 (&yr)[R3],
                                          f32x4 (&yi)[R3]) {
  static_assert(R3 == 1 || R3 == 2 || R3 == 4, "factors 1, i, -1, -i only");
  typedef MxT<kFP16> M;
  f16x8 xv[R3];
#pragma unroll
  for (int p = 0; p < R3; ++p)
    xv[p] = __builtin_bit_cast(f16x8, make_uint4(raw[p][0], raw[p][1], raw[p][2], raw[p][3]));
#pragma unroll
  for (int b = 0; b < R3; ++b) {
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 rp = z, rm = z, ip = z, im = z;
#pragma unroll
    for (int p = 0; p < R3; ++p) {
      // w^{b p} as a power of i
      const int q = (b * p * (4 / R3)) & 3;
      const f16x8 x = xv[p];
      if (q == 0) {
        rp = M::mma(A[b][1], x, M::mma(A[b][0], x, rp));
        ip = M::mma(A[b][3], x, M::mma(A[b][2], x, ip));
      } else if (q == 1) {
        rm = M::mma(A[b][3], x, M::mma(A[b][2], x, rm));
        ip = M::mma(A[b][1], x, M::mma(A[b][0], x, ip));
      } else if (q == 2) {
        rm = M::mma(A[b][1], x, M::mma(A[b][0], x, rm));
        im = M::mma(A[b][3], x, M::mma(A[b][2], x, im));
      } else {
        rp = M::mma(A[b][3], x, M::mma(A[b][2], x, rp));
        im = M::mma(A[b][1], x, M::mma(A[b][0], x, im));
      }
    }
    yr[b] = rp - rm;
    yi[b] = ip - im;
  }
}

}  // namespace ci
