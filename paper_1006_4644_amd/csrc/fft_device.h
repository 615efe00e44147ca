// fft_device.h -- register/LDS building blocks of the inverse transform.
//
// The correlator of eq. (matchedfilter) is taken back to the time domain by
// an unnormalised inverse DFT, z_j = sum_k Z_k w^{jk}, w = exp(+2 pi i/N)
// (the paper's device_cufft_C2R step).  On gfx950 it is a four-step
// transform N = N1 x N2 whose column DFTs (length L = 256 .. 2048) run
// inside one workgroup: 16 complex values per lane, radix-16 register
// butterflies, and Stockham exchanges through LDS between stages.
//
// Column DFT of length L = 256 R3 over NC interleaved columns (lane (c, t),
// c fastest, t in [0, L/16)):
//   stage 1: lane t holds X[t + (L/16) m], m = 0..15; radix 16 over m,
//            twiddle w_L^{a t};
//   stage 2: lane (a0, s2) = (t / R3, t % R3) holds the stage-1 outputs of
//            row a0 at s = s2 + R3 q; radix 16 over q, twiddle
//            w_{16 R3}^{a2 s2};
//   stage 3: lane t holds rows d = t + (L/16) i of the radix-R3 step;
//            output b lands at j = d + 256 b.
// R3 == 1 stops after stage 2 with outputs j = t + 16 a2.
// The LDS exchanges are laid out so that the lanes of one access hit
// distinct banks: exchange 1 pads its rows, exchange 2 rotates row d by d
// (by d/2 when R3 == 2).
#pragma once

#include <hip/hip_runtime.h>

namespace ci {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * (+i)
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }
// a * (-i)
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }

// 4-point inverse DFT in place: y_a = sum_q x_q i^{aq}.
__device__ __forceinline__ void idft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 a = cadd(x0, x2), b = csub(x0, x2);
  const float2 c = cadd(x1, x3), d = csub(x1, x3);
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, mul_i(d));
  x3 = csub(b, mul_i(d));
}

// 4-point inverse DFT of (x0, x1, 0, 0).
__device__ __forceinline__ void idft4_half(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 a = x0, d = x1;
  x0 = cadd(a, d);
  x2 = csub(a, d);
  x1 = cadd(a, mul_i(d));
  x3 = csub(a, mul_i(d));
}

__device__ __forceinline__ void idft2(float2& x0, float2& x1) {
  const float2 a = x0;
  x0 = cadd(a, x1);
  x1 = csub(a, x1);
}

// Multiply by w16^e = exp(2 pi i e / 16) for a compile-time e.
template <int E>
__device__ __forceinline__ float2 tw16(float2 v) {
  constexpr int e = E & 15;
  constexpr float C1 = 0.92387953251128674f;  // cos(pi/8)
  constexpr float S1 = 0.38268343236508977f;  // sin(pi/8)
  constexpr float R2 = 0.70710678118654752f;  // 1/sqrt(2)
  if constexpr (e == 0) return v;
  else if constexpr (e == 4) return mul_i(v);
  else if constexpr (e == 8) return make_float2(-v.x, -v.y);
  else if constexpr (e == 12) return mul_mi(v);
  else if constexpr (e == 2) return make_float2((v.x - v.y) * R2, (v.x + v.y) * R2);
  else if constexpr (e == 6) return make_float2(-(v.x + v.y) * R2, (v.x - v.y) * R2);
  else if constexpr (e == 10) return make_float2((v.y - v.x) * R2, -(v.x + v.y) * R2);
  else if constexpr (e == 14) return make_float2((v.x + v.y) * R2, (v.y - v.x) * R2);
  else {
    constexpr float cs[16] = {1.f, C1, R2, S1, 0.f, -S1, -R2, -C1,
                              -1.f, -C1, -R2, -S1, 0.f, S1, R2, C1};
    constexpr float c = cs[e], s = cs[(e + 12) & 15];  // sin(t) = cos(t - pi/2)
    return cmul(v, make_float2(c, s));
  }
}

// 16-point inverse DFT in place, X_a = sum_q x_q w16^{aq}, as 4 x 4:
// q = q1 + 4 q2, a = a1 + 4 a2.  Q: only x_q with q < Q can be nonzero (the
// others are not read); Q = 16 is the full transform.
template <int Q = 16>
__device__ __forceinline__ void idft16(float2 (&x)[16]) {
  static_assert(Q == 2 || Q == 4 || Q == 8 || Q == 16, "Q in {2, 4, 8, 16}");
  constexpr int NQ1 = Q < 4 ? Q : 4;  // rows q1 that can be nonzero
  float2 A[4][4];                      // A[q1][a1]
#pragma unroll
  for (int q1 = 0; q1 < NQ1; ++q1) {
    if constexpr (Q >= 8) {
      float2 y0 = x[q1], y1 = x[q1 + 4], y2, y3;
      if constexpr (Q == 8) {
        idft4_half(y0, y1, y2, y3);
      } else {
        y2 = x[q1 + 8];
        y3 = x[q1 + 12];
        idft4(y0, y1, y2, y3);
      }
      A[q1][0] = y0; A[q1][1] = y1; A[q1][2] = y2; A[q1][3] = y3;
    } else {
      A[q1][0] = A[q1][1] = A[q1][2] = A[q1][3] = x[q1];  // only q2 = 0
    }
  }
  A[1][1] = tw16<1>(A[1][1]); A[1][2] = tw16<2>(A[1][2]); A[1][3] = tw16<3>(A[1][3]);
  if constexpr (NQ1 > 2) {
    A[2][1] = tw16<2>(A[2][1]); A[2][2] = tw16<4>(A[2][2]); A[2][3] = tw16<6>(A[2][3]);
    A[3][1] = tw16<3>(A[3][1]); A[3][2] = tw16<6>(A[3][2]); A[3][3] = tw16<9>(A[3][3]);
  }
#pragma unroll
  for (int a1 = 0; a1 < 4; ++a1) {
    float2 y0 = A[0][a1], y1 = A[1][a1], y2, y3;
    if constexpr (NQ1 > 2) {
      y2 = A[2][a1];
      y3 = A[3][a1];
      idft4(y0, y1, y2, y3);
    } else {
      idft4_half(y0, y1, y2, y3);
    }
    x[a1] = y0; x[a1 + 4] = y1; x[a1 + 8] = y2; x[a1 + 12] = y3;
  }
}

// 8-point inverse DFT on x[O .. O+7]: q = q1 + 2 q2, a = a1 + 4 a2.
template <int O>
__device__ __forceinline__ void idft8(float2 (&x)[16]) {
  float2 e0 = x[O + 0], e1 = x[O + 2], e2 = x[O + 4], e3 = x[O + 6];
  float2 o0 = x[O + 1], o1 = x[O + 3], o2 = x[O + 5], o3 = x[O + 7];
  idft4(e0, e1, e2, e3);
  idft4(o0, o1, o2, o3);
  o1 = tw16<2>(o1);  // w8^1
  o2 = mul_i(o2);    // w8^2
  o3 = tw16<6>(o3);  // w8^3
  x[O + 0] = cadd(e0, o0); x[O + 4] = csub(e0, o0);
  x[O + 1] = cadd(e1, o1); x[O + 5] = csub(e1, o1);
  x[O + 2] = cadd(e2, o2); x[O + 6] = csub(e2, o2);
  x[O + 3] = cadd(e3, o3); x[O + 7] = csub(e3, o3);
}

// Radix-R3 DFTs on the 16/R3 groups x[i R3 .. i R3 + R3).
template <int R3>
__device__ __forceinline__ void idft_groups(float2 (&x)[16]) {
  if constexpr (R3 == 2) {
#pragma unroll
    for (int i = 0; i < 8; ++i) idft2(x[2 * i], x[2 * i + 1]);
  } else if constexpr (R3 == 4) {
#pragma unroll
    for (int i = 0; i < 4; ++i) idft4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]);
  } else if constexpr (R3 == 8) {
    idft8<0>(x);
    idft8<8>(x);
  }
}

// ---------------------------------------------------------------------------
// the column transform, stage by stage
// ---------------------------------------------------------------------------

// Every LDS access below is a per-lane base pointer plus a compile-time
// offset, so the address arithmetic costs a few instructions per stage.
// Exchange 1 pads its 16 rows to S1 = L/16 + P1 slots; exchange 2 rotates
// row d by d (or d/2 when R3 == 2), which is constant per lane.
template <int L, int NC>
struct Col {
  static constexpr int Lp = L / 16;
  static constexpr int R3 = L / 256;
  static constexpr int P1 = R3 == 1 ? 1 : (R3 == 2 ? 2 : (NC == 4 ? 4 : 0));
  static constexpr int S1 = Lp + P1;
  static constexpr int LDS_ELEMS = (16 * S1 > L ? 16 * S1 : L) * NC;
  static_assert(R3 == 1 || R3 == 2 || R3 == 4 || R3 == 8, "L in 256..2048");

  // Stage 1: radix 16 in registers (inputs m >= Q are zero), table twiddle
  // w_L^{a t}, store row a, position t.
  // tw: w_{L TS}^e at tw[e] (TS = 2048 / L for the global w_2048 table,
  // 1 for an LDS copy of w_L).
  template <int Q, int TS = 2048 / L>
  __device__ static __forceinline__ void stage1(float2 (&x)[16], float2* lds, unsigned t,
                                                unsigned c, const float2* tw) {
    idft16<Q>(x);
    // twiddle index a t TS, walked as a byte offset
    const char* twb = reinterpret_cast<const char*>(tw);
    const unsigned step = t * (unsigned)TS * (unsigned)sizeof(float2);
    unsigned off = 0;
#pragma unroll
    for (int a = 1; a < 16; ++a) {
      off += step;
      x[a] = cmul(x[a], *reinterpret_cast<const float2*>(twb + off));
    }
    float2* p = lds + t * NC + c;
#pragma unroll
    for (int a = 0; a < 16; ++a) p[a * S1 * NC] = x[a];
    __syncthreads();
  }

  // Stage 2 load (row a0 = t / R3, positions s2 + R3 q) and radix 16.
  __device__ static __forceinline__ void stage2(float2 (&x)[16], const float2* lds, unsigned t,
                                                unsigned c) {
    const unsigned a0 = t / R3, s2 = t % R3;
    const float2* p = lds + (a0 * S1 + s2) * NC + c;
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = p[q * R3 * NC];
    idft16(x);
  }

  // Stage-2 table twiddle w_{16 R3}^{a2 s2} = w_L^{16 a2 s2} (R3 > 1).
  template <int TS = 2048 / L>
  __device__ static __forceinline__ void stage2_twiddle(float2 (&x)[16], unsigned t,
                                                        const float2* tw) {
    if constexpr (R3 > 1) {
      const char* twb = reinterpret_cast<const char*>(tw);
      const unsigned step = (t % R3) * 16u * (unsigned)TS * (unsigned)sizeof(float2);
      unsigned off = 0;
#pragma unroll
      for (int a2 = 1; a2 < 16; ++a2) {
        off += step;
        x[a2] = cmul(x[a2], *reinterpret_cast<const float2*>(twb + off));
      }
    }
  }

  // Stage 3 (R3 > 1): store stage-2 outputs (row d = a0 + 16 a2, position
  // s2), reload rows d = t + Lp i, radix R3.
  __device__ static __forceinline__ void stage3(float2 (&x)[16], float2* lds, unsigned t,
                                                unsigned c) {
    if constexpr (R3 > 1) {
      const unsigned a0 = t / R3, s2 = t % R3;
      const unsigned rw = R3 == 2 ? ((s2 + (a0 >> 1)) & 1u) : ((s2 + a0) & (R3 - 1));
      __syncthreads();
      float2* pw = lds + (a0 * R3 + rw) * NC + c;
#pragma unroll
      for (int a2 = 0; a2 < 16; ++a2) pw[a2 * 16 * R3 * NC] = x[a2];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < R3; ++s) {
        const unsigned rr = R3 == 2 ? ((s + (t >> 1)) & 1u) : ((s + t) & (R3 - 1));
        const float2* pr = lds + (t * R3 + rr) * NC + c;
#pragma unroll
        for (int i = 0; i < 16 / R3; ++i) x[i * R3 + s] = pr[i * Lp * R3 * NC];
      }
      idft_groups<R3>(x);
    }
  }

  // Output index j in [0, L) held in register r, relative to lane t:
  // j = t + off(r).
  __host__ __device__ static constexpr int off(int r) {
    if constexpr (R3 == 1) return 16 * r;
    else return Lp * (r / R3) + 256 * (r % R3);
  }
  __device__ static __forceinline__ int out(int t, int r) { return t + off(r); }
  // Register holding the k-th smallest output of a lane.
  __host__ __device__ static constexpr int reg_by_order(int k) {
    if constexpr (R3 == 1) return k;
    else return (k % (16 / R3)) * R3 + k / (16 / R3);
  }
};

// Full column DFT with table twiddles (pass 2): see Col<L, NC>.  TS as in
// Col::stage1.
template <int L, int NC, int TS = 2048 / L>
__device__ __forceinline__ void fft_col(float2 (&x)[16], float2* lds, unsigned t, unsigned c,
                                        const float2* tw) {
  using K = Col<L, NC>;
  K::template stage1<16, TS>(x, lds, t, c, tw);
  K::stage2(x, lds, t, c);
  K::template stage2_twiddle<TS>(x, t, tw);
  K::stage3(x, lds, t, c);
}

}  // namespace ci
