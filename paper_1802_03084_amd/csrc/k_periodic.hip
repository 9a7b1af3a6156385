// Periodicity search (Law et al. 2018, section 3.1 footnote: a time segment is
// Fourier transformed to frequencies and each frequency is imaged; Figure 2
// caption: a modification of the innermost loop).
//
// Per DM trial:
//   1. k_time_fft_n (T = 64 .. 2048; k_time_fft, radix-2 in LDS, otherwise):
//      the dedispersed Stokes I series of COLS adjacent (baseline, channel)
//      pairs (zero past the end of the segment) is transformed along time
//      (forward, exp(-2 pi i f t / T), float32, twiddles from a float64
//      table) and frequencies f = 1 .. T/2 are written divided by T, rows of
//      (baseline, channel) so the gridding reads them contiguously.
//   2. Per batch of frequencies, k_grid_pf sums each occupied cell's
//      contributors (the plan's cell-sorted order, fixed summation order) into
//      one dense grid per frequency.  The dense imaging kernels transform it
//      as one complex image (the pair transform of (G, -iG): Re and Im are
//      the real images of G and -iG) and write its amplitude |I|.
//   3. The dense search kernel takes the amplitude image's peak and exact
//      lower median and thresholds peak / (median / sqrt(2 ln 2)).
// The transform length is the segment length, a power of two up to 8192.
#pragma clang fp contract(off)

#include "rf_internal.h"
#include "fft.h"

#include <hip/hip_fp16.h>

#include <algorithm>
#include <climits>

namespace {

constexpr int kThreads = 256;
constexpr int kLdsPoints = 8192;          // complex points per workgroup (64 KB)
// bytes of grids and images per frequency batch: enough frequencies that the
// per-image search (one workgroup per image) fills the 256 CUs
constexpr size_t kBatchBudget = (size_t)10 << 30;
constexpr float kInvRayleighMedian = 0.84932180028801907f;  // 1 / sqrt(2 ln 2)

constexpr size_t kAlign = 256;
inline size_t aup(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// tw[m] = exp(+2 pi i m / T), m < T, from float64
__global__ void k_time_twiddles(float2 *__restrict__ tw, int T) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)T, &s, &c);
  tw[k] = make_float2((float)c, (float)s);
}

__device__ __forceinline__ float2 load_c(const float2 *p, size_t i) { return p[i]; }
__device__ __forceinline__ float2 load_c(const __half2 *p, size_t i) {
  return __half22float2(p[i]);
}

// Lengths 64 .. 2048: the forward transform as the conjugate of the inverse
// transform of the conjugate input, with the register/LDS FFT of the image
// columns (ColFft<T>, COLS adjacent (baseline, channel) series per
// workgroup, tiles dealt to the XCDs in contiguous runs so neighbouring tiles
// share cache lines).  Each thread's series is tid mod COLS in every pass
// (NT is a multiple of COLS), so its delay and output column are fixed.
template <int T, typename E, int P>
__global__ __launch_bounds__(rf::ColCfg<T>::NT) void k_time_fft_n(
    const E *__restrict__ vis, float2 *__restrict__ out, const int32_t *__restrict__ delay,
    const float2 *__restrict__ tw, int nbc, int nchan) {
  using namespace rf;
  constexpr int COLS = ColCfg<T>::COLS, NT = ColCfg<T>::NT, S = ColCfg<T>::STRIDE;
  static_assert(NT % COLS == 0, "a thread's series must be the same in every pass");
  __shared__ float2 buf[COLS * S];
  const int ntile = (nbc + COLS - 1) / COLS;
  const int per = (ntile + 7) >> 3;
  const int b = blockIdx.x;
  const int L = (b & 7) * per + (b >> 3);
  if ((b >> 3) >= per || L >= ntile) return;
  const int tid = threadIdx.x;
  const int bc_raw = L * COLS + tid % COLS;
  const bool col_ok = bc_raw < nbc;
  const int bc = col_ok ? bc_raw : nbc - 1;
  const int d = delay[bc % nchan];
  const float inv_t = 1.0f / (float)T;
  fft_inverse<ColFft<T>, COLS, NT, S, false>(
      buf, tw, tid,
      [&](int, int i) {  // conjugate of the dedispersed Stokes I at time i
        const int src = i + d;
        const size_t e = ((size_t)min(src, T - 1) * nbc + bc) * P;
        float2 v;
        if (P == 2) {
          const float2 a = load_c(vis, e), q = load_c(vis, e + 1);
          v = make_float2((a.x + q.x) * 0.5f, (a.y + q.y) * 0.5f);
        } else {
          v = load_c(vis, e);
        }
        return (src < T && col_ok) ? make_float2(v.x, -v.y) : make_float2(0.f, 0.f);
      },
      [&](int, int y, float2 v) {  // frequency y = 1 .. T/2, conjugated back, over T
        if (y >= 1 && y <= T / 2 && col_ok)
          out[(size_t)(y - 1) * nbc + bc] = make_float2(v.x * inv_t, -v.y * inv_t);
      });
}

template <typename E, int P>
__global__ __launch_bounds__(kThreads) void k_time_fft(const E *__restrict__ vis,
                                                       float2 *__restrict__ out,
                                                       const int32_t *__restrict__ delay,
                                                       const float2 *__restrict__ tw, int T,
                                                       int log2t, int nbc, int nchan, int cols) {
  __shared__ float2 lds[kLdsPoints];  // [T][cols], T * cols == kLdsPoints
  const int bc0 = blockIdx.x * cols;
  const int tid = threadIdx.x;
  const int npts = T * cols;
  // load: dedispersed Stokes I at bit-reversed time positions
  for (int idx = tid; idx < npts; idx += kThreads) {
    const int t = idx / cols, col = idx - t * cols;
    const int bc = bc0 + col;
    float2 v = make_float2(0.f, 0.f);
    if (bc < nbc) {
      const int src = t + delay[bc % nchan];
      if (src < T) {
        const size_t e = ((size_t)src * nbc + bc) * P;
        if (P == 2) {
          const float2 a = load_c(vis, e), b = load_c(vis, e + 1);
          v = make_float2((a.x + b.x) * 0.5f, (a.y + b.y) * 0.5f);
        } else {
          v = load_c(vis, e);
        }
      }
    }
    const int r = (int)(__builtin_bitreverse32((uint32_t)t) >> (32 - log2t));
    lds[r * cols + col] = v;
  }
  __syncthreads();
  // radix-2 decimation in time, in place
  const int nbf = (T / 2) * cols;
  for (int s = 0; s < log2t; ++s) {
    const int half = 1 << s;
    const int tstep = T >> (s + 1);  // twiddle index stride
    for (int item = tid; item < nbf; item += kThreads) {
      const int b = item / cols, col = item - b * cols;
      const int j = b & (half - 1);
      const int i0 = ((b >> s) << (s + 1)) + j;
      const int i1 = i0 + half;
      const float2 wp = tw[j * tstep];  // the forward transform uses exp(-i): conjugate
      const float2 w = make_float2(wp.x, -wp.y);
      const float2 x = lds[i0 * cols + col], y = lds[i1 * cols + col];
      const float2 wy = make_float2(w.x * y.x - w.y * y.y, w.x * y.y + w.y * y.x);
      lds[i0 * cols + col] = make_float2(x.x + wy.x, x.y + wy.y);
      lds[i1 * cols + col] = make_float2(x.x - wy.x, x.y - wy.y);
    }
    __syncthreads();
  }
  // frequencies 1 .. T/2, divided by T
  const float inv_t = 1.0f / (float)T;
  const int nout = (T / 2) * cols;
  for (int idx = tid; idx < nout; idx += kThreads) {
    const int f = idx / cols + 1, col = idx - (f - 1) * cols;
    const int bc = bc0 + col;
    if (bc < nbc) {
      const float2 v = lds[f * cols + col];
      out[(size_t)(f - 1) * nbc + bc] = make_float2(v.x * inv_t, v.y * inv_t);
    }
  }
}

// Grid of each frequency row [0, nf) of F (rows of nbc values): only the
// occupied cells are written (the rest of the grids stays zero from the
// clear at the start of the search: every frequency occupies the same cells).
__global__ __launch_bounds__(kThreads) void k_grid_pf(const float2 *__restrict__ F, int nbc,
                                                      const int32_t *__restrict__ ucell,
                                                      const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ contrib,
                                                      int n_cells, int blocks_per_f, size_t npix2,
                                                      float2 *__restrict__ grid) {
  const int n = blockIdx.x / blocks_per_f;
  const int u = (blockIdx.x % blocks_per_f) * kThreads + threadIdx.x;
  if (u >= n_cells) return;
  const float2 *row = F + (size_t)n * nbc;
  float2 acc = make_float2(0.f, 0.f);
  const int e = off[u + 1];
  for (int q = off[u]; q < e; ++q) {
    const float2 v = row[contrib[q]];
    acc.x += v.x;
    acc.y += v.y;
  }
  grid[(size_t)n * npix2 + ucell[u]] = acc;
}

struct PLayout {
  size_t tw, F, grid, amp, imgws, total;
  int nf;
};

PLayout periodic_layout(const rf_plan *p) {
  PLayout L{};
  const int T = p->nint;
  const size_t n2 = (size_t)p->npix * p->npix;
  const size_t nbc = (size_t)p->nbl * p->nchan;
  const size_t per_f = n2 * sizeof(float2) + n2 * sizeof(float) +
                       (size_t)p->n_rows * p->npix * sizeof(float2);
  L.nf = (int)std::max<size_t>(1, std::min<size_t>((size_t)T / 2, kBatchBudget / per_f));
  size_t o = 0;
  L.tw = o;
  o += aup(sizeof(float2) * (size_t)std::max(1, T));
  L.F = o;
  o += aup(sizeof(float2) * (size_t)(T / 2) * nbc);
  L.grid = o;
  o += aup(sizeof(float2) * n2 * L.nf);
  L.amp = o;
  o += aup(sizeof(float) * n2 * L.nf);
  L.imgws = o;
  o += aup(image_ws_bytes(p, 2 * L.nf));
  L.total = o;
  return L;
}

}  // namespace

namespace {

template <typename E, int P>
rf_status time_fft_e(const rf_plan *p, const E *vis, float2 *F, const int32_t *delay,
                     const float2 *tw, int T, int log2t, int nbc, int cols, int nblk,
                     hipStream_t s) {
  const int nchan = p->nchan;
#define RF_TFFT(TT)                                                                          \
  case TT: {                                                                                 \
    constexpr int C = rf::ColCfg<TT>::COLS;                                                 \
    const int ntile = (nbc + C - 1) / C;                                                     \
    k_time_fft_n<TT, E, P><<<(unsigned)((ntile + 7) / 8 * 8), rf::ColCfg<TT>::NT, 0, s>>>( \
        vis, F, delay, tw, nbc, nchan);                                                      \
    break;                                                                                   \
  }
  switch (T) {
    RF_TFFT(64)
    RF_TFFT(128)
    RF_TFFT(256)
    RF_TFFT(512)
    RF_TFFT(1024)
    RF_TFFT(2048)
    default:
      k_time_fft<E, P><<<nblk, kThreads, 0, s>>>(vis, F, delay, tw, T, log2t, nbc, nchan, cols);
  }
#undef RF_TFFT
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

rf_status time_fft(const rf_plan *p, const void *vis, float2 *F, const int32_t *delay,
                   const float2 *tw, int T, int log2t, int nbc, int cols, int nblk,
                   hipStream_t s) {
  if (p->vis_dtype == RF_CF32)
    return p->npol == 2
               ? time_fft_e<float2, 2>(p, (const float2 *)vis, F, delay, tw, T, log2t, nbc, cols,
                                       nblk, s)
               : time_fft_e<float2, 1>(p, (const float2 *)vis, F, delay, tw, T, log2t, nbc, cols,
                                       nblk, s);
  return p->npol == 2
             ? time_fft_e<__half2, 2>(p, (const __half2 *)vis, F, delay, tw, T, log2t, nbc, cols,
                                      nblk, s)
             : time_fft_e<__half2, 1>(p, (const __half2 *)vis, F, delay, tw, T, log2t, nbc, cols,
                                      nblk, s);
}

}  // namespace

size_t periodic_ws_bytes(const rf_plan *p) { return periodic_layout(p).total; }

rf_status run_periodic(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                       int32_t *ncand, rf_image_stats *stats, void *ws, hipStream_t s) {
  const PLayout L = periodic_layout(p);
  char *base = (char *)ws;
  float2 *tw = (float2 *)(base + L.tw);
  float2 *F = (float2 *)(base + L.F);
  float2 *grid = (float2 *)(base + L.grid);
  float *amp = (float *)(base + L.amp);
  float2 *imgws = (float2 *)(base + L.imgws);
  const int T = p->nint;
  int log2t = 0;
  while ((1 << log2t) < T) ++log2t;
  const int cols = kLdsPoints / T;
  const int nbc = p->nbl * p->nchan;
  const size_t n2 = (size_t)p->npix * p->npix;
  const int nfreq = T / 2;

  rf_status st = launch_zero_i32(ncand, 1, s);
  if (st != RF_OK) return st;
  st = launch_zero_f32((float *)grid, 2 * n2 * (size_t)L.nf, s);  // unoccupied cells stay zero
  if (st != RF_OK) return st;
  k_time_twiddles<<<(T + kThreads - 1) / kThreads, kThreads, 0, s>>>(tw, T);
  RF_HIP_TRY(hipGetLastError());
  const int nblk = (nbc + cols - 1) / cols;
  const int bpf = (p->n_cells + kThreads - 1) / kThreads;
  const int no_window_lo = INT32_MIN, no_window_hi = INT32_MAX;
  for (int i = 0; i < p->ndm; ++i) {
    const int32_t *delay = p->d_delay + (size_t)i * p->nchan;
    st = time_fft(p, vis, F, delay, tw, T, log2t, nbc, cols, nblk, s);
    if (st != RF_OK) return st;
    for (int f0 = 0; f0 < nfreq; f0 += L.nf) {
      const int nf = std::min(L.nf, nfreq - f0);
      if (p->n_cells > 0) {
        k_grid_pf<<<(unsigned)(bpf * nf), kThreads, 0, s>>>(F + (size_t)f0 * nbc, nbc, p->d_ucell,
                                                            p->d_ucell_off, p->d_contrib,
                                                            p->n_cells, bpf, n2, grid);
        RF_HIP_TRY(hipGetLastError());
      }
      st = launch_image_amplitude(p, grid, nf, amp, imgws, s);
      if (st != RF_OK) return st;
      // image n of the batch is frequency f0 + 1 + n: tag t_int = f
      const rf_tag_gen gen{i, -1, 1, f0 + 1};
      rf_image_stats *st_out = stats ? stats + (size_t)i * nfreq + f0 : nullptr;
      st = launch_search_ex(p, amp, nf, nullptr, &gen, st_out, cand, cap, ncand,
                            kInvRayleighMedian, no_window_lo, no_window_hi, s);
      if (st != RF_OK) return st;
    }
  }
  return RF_OK;
}
