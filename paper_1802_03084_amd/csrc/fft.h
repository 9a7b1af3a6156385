// Workgroup-cooperative inverse FFTs (Stockham autosort, radix 8/16/32).
//
// A workgroup transforms F independent length-N sequences.  A pass of radix R
// (with NS = product of the earlier radices) performs, for every butterfly j
// in [0, N/R):
//   v[r] = x[j + r N/R] * w^(r (j mod NS)),  w = exp(+2 pi i / (NS R))
//   v    = DFT_R(v)            (inverse sign, natural order)
//   y[(j / NS) NS R + (j mod NS) + r NS] = v[r]
// which is the classical self-sorting Stockham formulation of the radix-R
// Cooley-Tukey FFT: after the last pass y is the inverse DFT in natural
// order.  A shape type fixes the radices (two or three passes held in
// registers): the first pass reads its inputs from wherever the caller keeps
// them (global memory for the column transform), the passes exchange through
// one padded LDS buffer, and the last pass hands its outputs to the caller in
// registers.  A butterfly's twiddles are the powers of one value of the table
// tw[m] = exp(+2 pi i m / N) (computed on the host in float64), formed in
// registers; each thread loads its table values once, before any barrier.
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

// x * exp(+2 pi i e / 32).  e is a compile-time constant at every call site
// after unrolling, so the switch folds away and trivial rotations cost nothing.
__device__ __forceinline__ float2 rot32(float2 x, int e) {
#pragma clang fp contract(off)
  constexpr float c1 = 0.98078528040323044913f;  // cos(pi/16)
  constexpr float s1 = 0.19509032201612826785f;  // sin(pi/16)
  constexpr float c2 = 0.92387953251128675613f;  // cos(pi/8)
  constexpr float s2 = 0.38268343236508977173f;  // sin(pi/8)
  constexpr float c3 = 0.83146961230254523708f;  // cos(3pi/16)
  constexpr float s3 = 0.55557023301960222474f;  // sin(3pi/16)
  constexpr float h = 0.70710678118654752440f;   // cos(pi/4)
  switch (e & 31) {
    case 0: return x;
    case 1: return crot(x, c1, s1);
    case 2: return crot(x, c2, s2);
    case 3: return crot(x, c3, s3);
    case 4: return make_float2(h * (x.x - x.y), h * (x.x + x.y));
    case 5: return crot(x, s3, c3);
    case 6: return crot(x, s2, c2);
    case 7: return crot(x, s1, c1);
    case 8: return make_float2(-x.y, x.x);
    case 9: return crot(x, -s1, c1);
    case 10: return crot(x, -s2, c2);
    case 11: return crot(x, -s3, c3);
    case 12: return make_float2(-h * (x.x + x.y), h * (x.x - x.y));
    case 13: return crot(x, -c3, s3);
    case 14: return crot(x, -c2, s2);
    case 15: return crot(x, -c1, s1);
    case 16: return make_float2(-x.x, -x.y);
    case 17: return crot(x, -c1, -s1);
    case 18: return crot(x, -c2, -s2);
    case 19: return crot(x, -c3, -s3);
    case 20: return make_float2(h * (x.y - x.x), -h * (x.x + x.y));
    case 21: return crot(x, -s3, -c3);
    case 22: return crot(x, -s2, -c2);
    case 23: return crot(x, -s1, -c1);
    case 24: return make_float2(x.y, -x.x);
    case 25: return crot(x, s1, -c1);
    case 26: return crot(x, s2, -c2);
    case 27: return crot(x, s3, -c3);
    case 28: return make_float2(h * (x.x + x.y), h * (x.y - x.x));
    case 29: return crot(x, c3, -s3);
    case 30: return crot(x, c2, -s2);
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

// In-register inverse DFT of length R in {2, 4, 8, 16, 32}: bit-reversed
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
        const float2 b = rot32(t[i + k + len / 2], k * (32 / len));
        t[i + k] = cadd(a, b);
        t[i + k + len / 2] = csub(a, b);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}

// Padded LDS index: one spare element after every 2^PS (PS = log2 of the
// first radix), so that the stride-R writes of the first pass spread over
// the LDS banks instead of piling onto one.
template <int PS>
__device__ __forceinline__ int pidx(int i) { return i + (i >> PS); }

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Radix schedule of a length-N transform: R0 R1 R2 = N, R2 = 1 for two
// passes.  PADDED is the padded LDS length of one sequence.
template <int N_, int R0_, int R1_, int R2_>
struct FftShape {
  static constexpr int N = N_, R0 = R0_, R1 = R1_, R2 = R2_;
  static_assert(R0 * R1 * R2 == N, "radices multiply to N");
  static constexpr int PS = ilog2(R0);
  static constexpr int PADDED = N + (N >> PS);
};

// Row transforms (along u) and column transforms (along v).  From 512 up the
// passes are of radix up to 16, so that a thread holds at most 16 values and
// four waves per SIMD fit in the register file.
template <int N> struct RowFft;
template <> struct RowFft<64> : FftShape<64, 8, 8, 1> {};
template <> struct RowFft<128> : FftShape<128, 16, 8, 1> {};
template <> struct RowFft<256> : FftShape<256, 16, 16, 1> {};
template <> struct RowFft<512> : FftShape<512, 8, 8, 8> {};
template <> struct RowFft<1024> : FftShape<1024, 16, 8, 8> {};
template <> struct RowFft<2048> : FftShape<2048, 16, 16, 8> {};
template <int N> struct ColFft;
template <> struct ColFft<64> : FftShape<64, 8, 8, 1> {};
template <> struct ColFft<128> : FftShape<128, 16, 8, 1> {};
template <> struct ColFft<256> : FftShape<256, 16, 16, 1> {};
template <> struct ColFft<512> : FftShape<512, 8, 8, 8> {};
template <> struct ColFft<1024> : FftShape<1024, 16, 8, 8> {};
template <> struct ColFft<2048> : FftShape<2048, 16, 16, 8> {};

// Butterfly index -> (sequence f, butterfly j).  JF: j fastest across
// threads (rows: contiguous along the transform); otherwise f fastest
// (columns: neighbouring threads hold neighbouring columns).
template <int F, int NB, bool JF>
__device__ __forceinline__ void fj_of(int idx, int &f, int &j) {
  if (JF) {
    f = idx / NB;
    j = idx % NB;
  } else {
    f = idx % F;
    j = idx / F;
  }
}

// Powers t[r] = b^r, r < R (t[0] = 1), each the product of two lower powers
// (r = floor(r/2) + ceil(r/2)): at most log2 R products deep, so every power
// stays within a few ulp of exp(+2 pi i r m / N) when b is a table value.
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 b, float2 (&t)[R]) {
  t[0] = make_float2(1.f, 0.f);
  if constexpr (R > 1) t[1] = b;
#pragma unroll
  for (int r = 2; r < R; ++r) t[r] = cmul(t[r / 2], t[r - r / 2]);
}

// Twiddles.  A radix-R pass multiplies element r of butterfly j by
// w^(r (j mod NS)), w = exp(+2 pi i / (NS R)): the powers of one table value
// per butterfly, tw[(j mod NS) N / (NS R)] (tw[m] = exp(+2 pi i m / N)).  The
// second pass's twiddles are applied by the first pass as it stores (its
// output r is element p / NB1 of second-pass butterfly p mod NB1, p = j R0 +
// r; as NB1 = R0 R2 that element is j / R2 for every r and the butterfly's
// j mod R0 is r, so the first pass's R0 twiddles are the powers of
// tw[(j / R2) N / (R0 R1)]); the last pass of a three-pass shape applies
// its own.  A thread therefore needs one table value per butterfly it takes
// in the first pass and in the last, loaded once, ahead of every barrier.
template <class Sh, int F, int NT, bool JF>
struct TwBases {
  static constexpr int N = Sh::N;
  static constexpr int NB0 = N / Sh::R0, TOT0 = F * NB0, Q0 = (TOT0 + NT - 1) / NT;
  static constexpr bool THREE = Sh::R2 != 1;
  static constexpr int NBL = N / Sh::R2, TOTL = F * NBL, QL = THREE ? (TOTL + NT - 1) / NT : 1;
  float2 first[Q0];
  float2 last[QL];
  __device__ __forceinline__ void load(const float2 *__restrict__ tw, int tid) {
#pragma unroll
    for (int q = 0; q < Q0; ++q) {  // threads past the butterflies load a value they never use
      int f, j;
      fj_of<F, NB0, JF>(min(tid + q * NT, TOT0 - 1), f, j);
      first[q] = tw[(j / Sh::R2) * (N / (Sh::R0 * Sh::R1))];
    }
    if constexpr (THREE) {
      constexpr int NS = Sh::R0 * Sh::R1;
#pragma unroll
      for (int q = 0; q < QL; ++q) {
        int f, j;
        fj_of<F, NBL, JF>(min(tid + q * NT, TOTL - 1), f, j);
        last[q] = tw[(j % NS) * (N / (NS * Sh::R2))];
      }
    }
  }
};

// First pass: inputs from load(f, i), radix-R0 DFT, results (times the
// second pass's twiddles) to LDS at the Stockham position j R0 + r.  The
// pass comes in three parts (fft_first_load: the inputs into registers;
// fft_first_dft; fft_first_store: the LDS write) so that a caller can do
// other work while the loads are in flight.
template <class Sh, int F, int NT>
struct FirstRegs {
  static constexpr int R = Sh::R0, NB = Sh::N / R, TOT = F * NB, Q = (TOT + NT - 1) / NT;
  float2 v[Q][R];
};

template <class Sh, int F, int NT, bool JF, class Load>
__device__ __forceinline__ void fft_first_load(int tid, Load load, FirstRegs<Sh, F, NT> &x) {
  using X = FirstRegs<Sh, F, NT>;
#pragma unroll
  for (int q = 0; q < X::Q; ++q) {
    const int idx = tid + q * NT;
    if ((X::TOT % NT) == 0 || idx < X::TOT) {
      int f, j;
      fj_of<F, X::NB, JF>(idx, f, j);
#pragma unroll
      for (int r = 0; r < X::R; ++r) x.v[q][r] = load(f, j + r * X::NB);
    }
  }
}

template <class Sh, int F, int NT>
__device__ __forceinline__ void fft_first_dft(FirstRegs<Sh, F, NT> &x) {
  using X = FirstRegs<Sh, F, NT>;
#pragma unroll
  for (int q = 0; q < X::Q; ++q) dft<X::R>(x.v[q]);
}

// LDS write of the first pass, each output multiplied by the twiddle the
// second pass would apply to it; the caller synchronises before it (if buf is
// still being read) and after.
template <class Sh, int F, int NT, int S, bool JF>
__device__ __forceinline__ void fft_first_store(float2 *buf, const TwBases<Sh, F, NT, JF> &tb,
                                                int tid, FirstRegs<Sh, F, NT> &x) {
  using X = FirstRegs<Sh, F, NT>;
  constexpr int PS = Sh::PS;
#pragma unroll
  for (int q = 0; q < X::Q; ++q) {
    const int idx = tid + q * NT;
    if ((X::TOT % NT) == 0 || idx < X::TOT) {
      int f, j;
      fj_of<F, X::NB, JF>(idx, f, j);
      float2 t[X::R];
      twiddle_powers<X::R>(tb.first[q], t);
#pragma unroll
      for (int r = 0; r < X::R; ++r) buf[f * S + pidx<PS>(j * X::R + r)] = cmul(x.v[q][r], t[r]);
    }
  }
}

template <class Sh, int F, int NT, int S, bool JF, class Load>
__device__ __forceinline__ void fft_first(float2 *buf, const TwBases<Sh, F, NT, JF> &tb, int tid,
                                          Load load) {
  FirstRegs<Sh, F, NT> x;
  fft_first_load<Sh, F, NT, JF>(tid, load, x);
  __builtin_amdgcn_sched_barrier(0);  // every load issued before the transform starts
  fft_first_dft<Sh, F, NT>(x);
  __syncthreads();  // inputs may have come from buf
  fft_first_store<Sh, F, NT, S, JF>(buf, tb, tid, x);
  __syncthreads();
}

// Loads butterfly (f, j) of a radix-R pass from LDS; with TW, multiplies
// element r by base^r (every element, r = 0 included: by 1, exact up to the
// sign of a zero).
template <int N, int R, int S, int PS, bool TW>
__device__ __forceinline__ void fft_gather(const float2 *buf, float2 base, int f, int j,
                                           float2 (&v)[R]) {
  constexpr int NB = N / R;
  float2 t[R];
  if constexpr (TW) twiddle_powers<R>(base, t);
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = buf[f * S + pidx<PS>(j + r * NB)];
  if constexpr (TW) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = cmul(v[r], t[r]);
  }
}

// Middle pass (its twiddles were applied by the first pass): LDS -> LDS in place.
template <class Sh, int R, int NS, int F, int NT, int S, bool JF>
__device__ __forceinline__ void fft_mid(float2 *buf, int tid) {
  constexpr int N = Sh::N, NB = N / R, TOT = F * NB, Q = (TOT + NT - 1) / NT, PS = Sh::PS;
  float2 v[Q][R];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = tid + q * NT;
    if ((TOT % NT) == 0 || idx < TOT) {
      int f, j;
      fj_of<F, NB, JF>(idx, f, j);
      fft_gather<N, R, S, PS, false>(buf, make_float2(1.f, 0.f), f, j, v[q]);
      dft<R>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = tid + q * NT;
    if ((TOT % NT) == 0 || idx < TOT) {
      int f, j;
      fj_of<F, NB, JF>(idx, f, j);
      const int d0 = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[f * S + pidx<PS>(d0 + r * NS)] = v[q][r];
    }
  }
  __syncthreads();
}

// Last pass: LDS -> registers, results handed to store(f, k, value) with k the
// natural-order output index.  TW: the pass applies its own twiddles (the
// third pass of a three-pass shape), from the thread's bases.
template <class Sh, int R, int NS, int F, int NT, int S, bool JF, bool TW, class Store>
__device__ __forceinline__ void fft_last(const float2 *buf, const TwBases<Sh, F, NT, JF> &tb,
                                         int tid, Store store) {
  constexpr int N = Sh::N, NB = N / R, TOT = F * NB, Q = (TOT + NT - 1) / NT, PS = Sh::PS;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = tid + q * NT;
    if ((TOT % NT) == 0 || idx < TOT) {
      int f, j;
      fj_of<F, NB, JF>(idx, f, j);
      float2 v[R];
      fft_gather<N, R, S, PS, TW>(buf, tb.last[TW ? q : 0], f, j, v);
      dft<R>(v);
      const int d0 = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) store(f, d0 + r * NS, v[r]);
    }
  }
}

// Last pass variant: consume(f, k0, kstep, v) receives a butterfly's R outputs
// at natural-order indices k0 + r * kstep in increasing r (kstep = NS).
template <class Sh, int R, int NS, int F, int NT, int S, bool JF, bool TW, class Consume>
__device__ __forceinline__ void fft_last_block(const float2 *buf, const TwBases<Sh, F, NT, JF> &tb,
                                               int tid, Consume consume) {
  constexpr int N = Sh::N, NB = N / R, TOT = F * NB, Q = (TOT + NT - 1) / NT, PS = Sh::PS;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = tid + q * NT;
    if ((TOT % NT) == 0 || idx < TOT) {
      int f, j;
      fj_of<F, NB, JF>(idx, f, j);
      float2 v[R];
      fft_gather<N, R, S, PS, TW>(buf, tb.last[TW ? q : 0], f, j, v);
      dft<R>(v);
      consume(f, (j / NS) * NS * R + (j % NS), NS, v);
    }
  }
}

// The passes after the first (buf holds the first pass's output, written
// with fft_first_store and synchronised); the last pass hands whole
// butterflies to consume.
template <class Sh, int F, int NT, int S, bool JF, class Consume>
__device__ __forceinline__ void fft_rest_blocks(float2 *buf, const TwBases<Sh, F, NT, JF> &tb,
                                                int tid, Consume consume) {
  if constexpr (Sh::R2 == 1) {
    fft_last_block<Sh, Sh::R1, Sh::R0, F, NT, S, JF, false>(buf, tb, tid, consume);
  } else {
    fft_mid<Sh, Sh::R1, Sh::R0, F, NT, S, JF>(buf, tid);
    fft_last_block<Sh, Sh::R2, Sh::R0 * Sh::R1, F, NT, S, JF, true>(buf, tb, tid, consume);
  }
}

// Inverse (exp(+i)) unnormalised FFT of F sequences of length N: inputs from
// load(f, i), outputs to store(f, k, value), LDS buf of F * S elements
// (S >= Sh::PADDED) for the exchanges between passes; tb holds the thread's
// twiddle bases (TwBases::load), or the second form loads them first.
template <class Sh, int F, int NT, int S, bool JF, class Load, class Store>
__device__ __forceinline__ void fft_inverse(float2 *buf, const TwBases<Sh, F, NT, JF> &tb,
                                            int tid, Load load, Store store) {
  fft_first<Sh, F, NT, S, JF>(buf, tb, tid, load);
  if constexpr (Sh::R2 == 1) {
    fft_last<Sh, Sh::R1, Sh::R0, F, NT, S, JF, false>(buf, tb, tid, store);
  } else {
    fft_mid<Sh, Sh::R1, Sh::R0, F, NT, S, JF>(buf, tid);
    fft_last<Sh, Sh::R2, Sh::R0 * Sh::R1, F, NT, S, JF, true>(buf, tb, tid, store);
  }
}
template <class Sh, int F, int NT, int S, bool JF, class Load, class Store>
__device__ __forceinline__ void fft_inverse(float2 *buf, const float2 *__restrict__ tw, int tid,
                                            Load load, Store store) {
  TwBases<Sh, F, NT, JF> tb;
  tb.load(tw, tid);
  fft_inverse<Sh, F, NT, S, JF>(buf, tb, tid, load, store);
}

// Z value of the paired Hermitian transform at grid position (v, u), with the
// image normalisation folded in:
//   Z = s/(2W) [G_a(v,u) + conj G_a(-v,-u) + i (G_b(v,u) + conj G_b(-v,-u))]
// with s = (-1)^(u+v) and sg = s/(2W).  Evaluated as the (v,u) term plus the
// mirrored term in this fixed order, so that every caller (dense grids or
// gathered cells) produces bit-identical values.
__device__ __forceinline__ float2 zval(float2 a, float2 am, float2 b, float2 bm, float sg) {
#pragma clang fp contract(off)
  const float x = sg * (a.x - b.y) + sg * (am.x + bm.y);
  const float y = sg * (a.y + b.x) + sg * (bm.x - am.y);
  return make_float2(x, y);
}

// Raw buffer access: a load at an offset at or past the resource's size
// returns zero (the hardware range check), so a load is switched off by its
// offset alone and issued unconditionally, with no branch around it.
constexpr uint32_t kNoLoad = 0x7ffffff0u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           0x00020000);
}
// The same for a pointer and size that are uniform across the wave, read
// from its first lane so that the resource stays in scalar registers (a
// resource the compiler cannot prove uniform is used in a loop over the
// lanes' distinct values)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc_u(const void *p, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return buf_rsrc(reinterpret_cast<const void *>(((uint64_t)hi << 32) | lo),
                  __builtin_amdgcn_readfirstlane(bytes));
}
__device__ __forceinline__ float2 buf_load_f2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
__device__ __forceinline__ float4 buf_load_f4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
  return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                     __uint_as_float(v.w));
}
__device__ __forceinline__ float buf_load_f1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// Launch shapes of the two imaging passes for image side N.
template <int N>
struct RowCfg {  // dense rows: F grid rows per workgroup (4096 points: ~35 KB LDS)
  static constexpr int NT = 256;
  static constexpr int F = (4096 / N) < 64 ? (4096 / N) : 64;
  static constexpr int STRIDE = RowFft<N>::PADDED;
};
template <int N>
struct ColCfg {  // columns: COLS columns per workgroup
  // 4 columns from 1024 up (~35 KB LDS at 1024: four workgroups per CU,
  // whose load and transform phases interleave; ~70 KB at 2048), 8 at 512
  // (~37 KB), else 8192 points per workgroup
  static constexpr int COLS = N >= 1024 ? 4 : (N >= 512 ? 8 : 32 < N ? 32 : N);
  static constexpr int FIRST = COLS * N / ColFft<N>::R0;  // first-pass butterflies
  static constexpr int NT = N >= 512 ? (FIRST < 512 ? FIRST : 512) : (FIRST < 256 ? 256 : FIRST);
  // Columns vary fastest across lanes: a 64-bit LDS access serves 16 lanes
  // per cycle (COLS columns x 16/COLS butterflies), whose slots f STRIDE +
  // 17 j + r (first pass; the other passes alike) fall on distinct 8-byte
  // banks when STRIDE = 16/COLS modulo 16 (PADDED is a multiple of 16).
  static constexpr int STRIDE = ColFft<N>::PADDED + (COLS < 16 ? 16 / COLS : 1);
};

}  // namespace rf
