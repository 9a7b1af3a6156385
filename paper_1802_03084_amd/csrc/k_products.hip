// Second-tier candidate products (Law et al. 2018, section 3.1: candidates
// above a second, higher threshold, typically 7 sigma, get visualisations;
// section 3.3: the candidate's image and its spectrum).
//
// For one candidate (DM trial i, width w, resampled integration k, pixel
// (x, y)) the products are
//   * the cutout: the 2h x 2h window of the candidate's image centred on
//     (x, y), wrapping at the image edges (the image is an inverse DFT);
//   * the dynamic spectrum: rows k - nspec/2 .. k + nspec/2 - 1 (zero outside
//     the segment), each channel the mean over its gridded baselines of the
//     Stokes I sample turned to the pixel with the gridding's cell phases
//     exp(+2 pi i (iu (x - N/2) + iv (y - N/2)) / N), so that the channel sum
//     weighted by gridded baselines, over W, is the image pixel.
//
// Both start from one gather of the dedispersed, resampled integrations
// (k_gather_rs: the zero-filled shift then the decimating mean, summed in
// float32 in increasing order), threads along the contiguous (baseline,
// channel, polarisation) axis.  The image is formed from the centre row by
// the dense gridding and imaging kernels; the spectrum reduces over baselines
// with one thread per (row, channel), adjacent threads on adjacent channels
// so every baseline's loads are contiguous.  Products are few (the second
// tier is rare), so each candidate is processed in turn on the stream.
#include "rf_internal.h"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 load_c(const float2 *p, size_t i) { return p[i]; }
__device__ __forceinline__ float2 load_c(const __half2 *p, size_t i) {
  return __half22float2(p[i]);
}

template <typename E>
__global__ __launch_bounds__(kThreads) void k_gather_rs(const E *__restrict__ in,
                                                        float2 *__restrict__ out,
                                                        const int32_t *__restrict__ delay,
                                                        int nint, int nelem, int npol, int nchan,
                                                        int w, int k_first, int K) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= nelem) return;
  const int s = blockIdx.y;
  const int kk = k_first + s;
  float2 acc = make_float2(0.f, 0.f);
  if (kk >= 0 && kk < K) {
    const int d = delay[(e / npol) % nchan];
    for (int q = 0; q < w; ++q) {
      const int t = kk * w + q + d;
      if (t < nint) {
        const float2 x = load_c(in, (size_t)t * nelem + e);
        acc.x += x.x;
        acc.y += x.y;
      }
    }
    const float iw = 1.0f / (float)w;  // as the search's resampling
    acc.x *= iw;
    acc.y *= iw;
  }
  out[(size_t)s * nelem + e] = acc;
}

__global__ __launch_bounds__(kThreads) void k_cutout(const float *__restrict__ img,
                                                     float *__restrict__ out, int N, int x, int y,
                                                     int half) {
  const int side = 2 * half;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= side * side) return;
  const int r = i / side, q = i - r * side;
  const int row = (y - half + r) & (N - 1);
  const int col = (x - half + q) & (N - 1);
  out[i] = img[(size_t)row * N + col];
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_spectrum(const float2 *__restrict__ rs,
                                                       const int32_t *__restrict__ cells,
                                                       const float2 *__restrict__ tw,
                                                       float *__restrict__ spec, int nbl,
                                                       int nchan, int N, int dx, int dy) {
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= nchan) return;
  const int s = blockIdx.y;
  const float2 *row = rs + (size_t)s * nbl * nchan * P;
  const int lim = N / 2 - 1;
  float acc = 0.f;
  int cnt = 0;
  for (int b = 0; b < nbl; ++b) {
    const int bc = b * nchan + c;
    const int iu = cells[2 * bc], iv = cells[2 * bc + 1];
    if (iu < -lim || iu > lim || iv < -lim || iv > lim) continue;
    float2 vi;
    if (P == 2) {
      const float2 a = row[2 * (size_t)bc], z = row[2 * (size_t)bc + 1];
      vi = make_float2((a.x + z.x) * 0.5f, (a.y + z.y) * 0.5f);
    } else {
      vi = row[bc];
    }
    const float2 t = tw[(iu * dx + iv * dy) & (N - 1)];
    acc += vi.x * t.x - vi.y * t.y;
    ++cnt;
  }
  spec[(size_t)s * nchan + c] = cnt ? acc / (float)cnt : 0.f;
}

constexpr size_t kAlign = 256;
inline size_t aup(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

}  // namespace

size_t products_ws_bytes(const rf_plan *p, int nspec) {
  const size_t n2 = (size_t)p->npix * p->npix;
  const size_t nelem = (size_t)p->nbl * p->nchan * p->npol;
  return aup(sizeof(float2) * nelem * (size_t)nspec) + aup(sizeof(float2) * n2) +
         aup(sizeof(float) * n2) + aup(image_ws_bytes(p, 1));
}

rf_status run_products(const rf_plan *p, const void *vis, const rf_candidate *cand, int ncand,
                       int half, int nspec, float *cutout, float *spec, void *ws,
                       hipStream_t s) {
  const int N = p->npix;
  const size_t n2 = (size_t)N * N;
  const int nelem = p->nbl * p->nchan * p->npol;
  char *base = (char *)ws;
  float2 *rs = (float2 *)base;
  float2 *grid = (float2 *)(base + aup(sizeof(float2) * (size_t)nelem * nspec));
  float *img = (float *)((char *)grid + aup(sizeof(float2) * n2));
  float2 *img_ws = (float2 *)((char *)img + aup(sizeof(float) * n2));
  const int side = 2 * half;
  for (int n = 0; n < ncand; ++n) {
    const rf_candidate &cd = cand[n];
    const int w = p->width[cd.width_idx];
    const int k = cd.t_int / w;
    const int K = p->nint / w;
    const int32_t *delay = p->d_delay + (size_t)cd.dm_idx * p->nchan;
    const dim3 g((nelem + kThreads - 1) / kThreads, nspec);
    if (p->vis_dtype == RF_CF32)
      k_gather_rs<float2><<<g, kThreads, 0, s>>>((const float2 *)vis, rs, delay, p->nint, nelem,
                                                 p->npol, p->nchan, w, k - nspec / 2, K);
    else
      k_gather_rs<__half2><<<g, kThreads, 0, s>>>((const __half2 *)vis, rs, delay, p->nint, nelem,
                                                  p->npol, p->nchan, w, k - nspec / 2, K);
    RF_HIP_TRY(hipGetLastError());
    if (spec) {
      const dim3 gs((p->nchan + kThreads - 1) / kThreads, nspec);
      float *out = spec + (size_t)n * nspec * p->nchan;
      if (p->npol == 2)
        k_spectrum<2><<<gs, kThreads, 0, s>>>(rs, p->d_cells, p->d_tw, out, p->nbl, p->nchan, N,
                                              cd.x - N / 2, cd.y - N / 2);
      else
        k_spectrum<1><<<gs, kThreads, 0, s>>>(rs, p->d_cells, p->d_tw, out, p->nbl, p->nchan, N,
                                              cd.x - N / 2, cd.y - N / 2);
      RF_HIP_TRY(hipGetLastError());
    }
    if (cutout) {
      const float2 *centre = rs + (size_t)(nspec / 2) * nelem;
      rf_status st = launch_grid_dense(p, centre, 1, grid, s);
      if (st != RF_OK) return st;
      st = launch_image_dense(p, grid, 1, img, img_ws, s);
      if (st != RF_OK) return st;
      const int cells = side * side;
      k_cutout<<<(cells + kThreads - 1) / kThreads, kThreads, 0, s>>>(
          img, cutout + (size_t)n * cells, N, cd.x, cd.y, half);
      RF_HIP_TRY(hipGetLastError());
    }
  }
  return RF_OK;
}
