// Workgroup-cooperative inverse FFTs in LDS (Stockham autosort, radix 4/8/16).
//
// A workgroup transforms F independent length-N sequences held in LDS, each
// starting STRIDE complex elements after the previous one.  A pass of radix R
// (with NS = product of the earlier radices) performs, for every butterfly j
// in [0, N/R):
//   v[r] = x[j + r N/R] * w^(r (j mod NS)),  w = exp(+2 pi i / (NS R))
//   v    = DFT_R(v)            (inverse sign, natural order)
//   y[(j / NS) NS R + (j mod NS) + r NS] = v[r]
// which is the classical self-sorting Stockham formulation of the radix-R
// Cooley-Tukey FFT: after the last pass y is the inverse DFT in natural
// order.  Each thread loads all of its butterflies' inputs into registers
// before a barrier and writes them after it, so one LDS buffer suffices.
// Twiddles come from an LDS table tw[m] = exp(+2 pi i m / N) computed on the
// host in float64.
#pragma once

#include <hip/hip_runtime.h>

namespace rf {

// The arithmetic below fixes its own fused multiply-adds (contraction is off
// and fmaf is explicit), so every kernel that inlines these routines rounds
// identically: the fused and step-chain paths produce bit-identical images.
__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 crot(float2 x, float c, float s) {
#pragma clang fp contract(off)
  return make_float2(__builtin_fmaf(x.x, c, -(x.y * s)), __builtin_fmaf(x.x, s, x.y * c));
}

// x * exp(+2 pi i e / 16).  e is a compile-time constant at every call site
// after unrolling, so the switch folds away and trivial rotations cost nothing.
__device__ __forceinline__ float2 rot16(float2 x, int e) {
#pragma clang fp contract(off)
  constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
  constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
  constexpr float h = 0.70710678118654752440f;   // cos(pi/4)
  switch (e & 15) {
    case 0: return x;
    case 1: return crot(x, c1, s1);
    case 2: return make_float2(h * (x.x - x.y), h * (x.x + x.y));
    case 3: return crot(x, s1, c1);
    case 4: return make_float2(-x.y, x.x);
    case 5: return crot(x, -s1, c1);
    case 6: return make_float2(-h * (x.x + x.y), h * (x.x - x.y));
    case 7: return crot(x, -c1, s1);
    case 8: return make_float2(-x.x, -x.y);
    case 9: return crot(x, -c1, -s1);
    case 10: return make_float2(h * (x.y - x.x), -h * (x.x + x.y));
    case 11: return crot(x, -s1, -c1);
    case 12: return make_float2(x.y, -x.x);
    case 13: return crot(x, s1, -c1);
    case 14: return make_float2(h * (x.x + x.y), h * (x.y - x.x));
    default: return crot(x, c1, -s1);
  }
}

template <int R>
__device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register inverse DFT of length R in {2, 4, 8, 16}: bit-reversed
// radix-2 decimation in time, natural-order output.
template <int R>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  float2 t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[i] = v[bitrev<R>(i)];
#pragma unroll
  for (int len = 2; len <= R; len *= 2) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        const float2 a = t[i + k];
        const float2 b = rot16(t[i + k + len / 2], k * (16 / len));
        t[i + k] = cadd(a, b);
        t[i + k + len / 2] = csub(a, b);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}

// Padded LDS index: one spare element after every 2^PS, so that the stride-R
// writes of the first pass (and the strided column gathers) spread over the
// LDS banks instead of piling onto one.
template <int PS>
__device__ __forceinline__ int pidx(int i) { return i + (i >> PS); }

template <int N, int R, int NS, int F, int NT, int STRIDE, int PS>
__device__ __forceinline__ void stockham_pass(float2 *buf, const float2 *tw, int tid) {
  constexpr int NB = N / R;
  constexpr int TOT = F * NB;
  constexpr int Q = (TOT + NT - 1) / NT;
  float2 v[Q][R];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = tid + q * NT;
    if ((TOT % NT) == 0 || idx < TOT) {
      const int f = idx / NB, j = idx % NB;
      const float2 *src = buf + f * STRIDE;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[pidx<PS>(j + r * NB)];
      if (NS > 1) {
        const int jm = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[jm * r * (N / (NS * R))]);
      }
      dft<R>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = tid + q * NT;
    if ((TOT % NT) == 0 || idx < TOT) {
      const int f = idx / NB, j = idx % NB;
      float2 *dst = buf + f * STRIDE;
      const int d0 = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[pidx<PS>(d0 + r * NS)] = v[q][r];
    }
  }
  __syncthreads();
}

// Radix schedule and LDS padding for each supported N.
template <int N>
struct FftShape {
  static_assert(N >= 64 && N <= 2048 && (N & (N - 1)) == 0, "N must be 2^k in [64, 2048]");
  static constexpr int PS = (N == 512) ? 3 : 4;  // log2 of the first radix
  static constexpr int PADDED = N + (N >> PS);   // padded length of one sequence
};

// Inverse (exp(+i)) unnormalised FFT of F sequences of length N in LDS, each
// stored padded (element i at pidx(i)) from buf + f * STRIDE.  Callers
// synchronise before (inputs written) and may read after return.
template <int N, int F, int NT, int STRIDE>
__device__ __forceinline__ void fft_inverse(float2 *buf, const float2 *tw, int tid) {
  constexpr int PS = FftShape<N>::PS;
  if constexpr (N == 64) {
    stockham_pass<N, 16, 1, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 4, 16, F, NT, STRIDE, PS>(buf, tw, tid);
  } else if constexpr (N == 128) {
    stockham_pass<N, 16, 1, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 8, 16, F, NT, STRIDE, PS>(buf, tw, tid);
  } else if constexpr (N == 256) {
    stockham_pass<N, 16, 1, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 16, 16, F, NT, STRIDE, PS>(buf, tw, tid);
  } else if constexpr (N == 512) {
    stockham_pass<N, 8, 1, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 8, 8, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 8, 64, F, NT, STRIDE, PS>(buf, tw, tid);
  } else if constexpr (N == 1024) {
    stockham_pass<N, 16, 1, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 16, 16, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 4, 256, F, NT, STRIDE, PS>(buf, tw, tid);
  } else {
    stockham_pass<N, 16, 1, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 16, 16, F, NT, STRIDE, PS>(buf, tw, tid);
    stockham_pass<N, 8, 256, F, NT, STRIDE, PS>(buf, tw, tid);
  }
}

// Z value of the paired Hermitian transform at grid position (v, u):
//   Z = s/2 [G_a(v,u) + conj G_a(-v,-u) + i (G_b(v,u) + conj G_b(-v,-u))]
// with s = (-1)^(u+v) and sg = s/2.  Evaluated as the (v,u) term plus the
// mirrored term in this fixed order, so that every caller (dense grids or
// gathered cells) produces bit-identical values.
__device__ __forceinline__ float2 zval(float2 a, float2 am, float2 b, float2 bm, float sg) {
#pragma clang fp contract(off)
  const float x = sg * (a.x - b.y) + sg * (am.x + bm.y);
  const float y = sg * (a.y + b.x) + sg * (bm.x - am.y);
  return make_float2(x, y);
}

// Launch shapes of the two imaging passes for image side N.
template <int N>
struct RowCfg {
  static constexpr int NT = 512;
  static constexpr int F = (8192 / N) < 64 ? (8192 / N) : 64;  // rows per workgroup
  static constexpr int STRIDE = FftShape<N>::PADDED;
};
template <int N>
struct ColCfg {
  static constexpr int NT = 1024;
  static constexpr int COLS = (16384 / N) < N ? (16384 / N) : N;  // columns per workgroup
  static constexpr int STRIDE = FftShape<N>::PADDED + 1;          // odd: spreads the transpose
};

// Column tile of the row-transformed data: buf[x][pidx(v)] = M[slot(v)][x0 + x]
// (zero for rows without samples), COLS columns.  The trip count is a
// compile-time constant so every thread issues all of its loads before it
// stores any of them.
template <int N>
__device__ __forceinline__ void load_col_tile(const float2 *__restrict__ Mp,
                                              const int32_t *__restrict__ row_slot, float2 *buf,
                                              int tid) {
  constexpr int COLS = ColCfg<N>::COLS, NT = ColCfg<N>::NT, S = ColCfg<N>::STRIDE;
  constexpr int PS = FftShape<N>::PS;
  constexpr int Q = (N * COLS + NT - 1) / NT;
  float2 v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = tid + q * NT;
    v[q] = make_float2(0.f, 0.f);
    if ((N * COLS) % NT == 0 || e < N * COLS) {
      const int slot = row_slot[e / COLS];
      if (slot >= 0) v[q] = Mp[(size_t)slot * N + e % COLS];
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = tid + q * NT;
    if ((N * COLS) % NT == 0 || e < N * COLS) buf[(e % COLS) * S + pidx<PS>(e / COLS)] = v[q];
  }
}

}  // namespace rf
