// Stokes I and nearest-cell gridding onto a dense N x N grid.
//
// Stokes I is the mean of the two polarisations (Law et al. 2018, section 3.1:
// a Stokes I image per DM and width).  Gridding is the reading used for the
// paper's unstated step: unit weights, nearest cell, no convolution kernel.
// The plan holds the pairs sorted by (cell, pair), so each occupied cell is a
// contiguous run of contributors and one thread sums it in a fixed order: no
// atomics, bit-reproducible from run to run.
#include "rf_internal.h"

#include <algorithm>

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_fill_zero(float4 *__restrict__ p, size_t n4) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_grid_cells(
    const float2 *__restrict__ vis, int nbc, const int32_t *__restrict__ ucell,
    const int32_t *__restrict__ off, const int32_t *__restrict__ contrib, int n_cells,
    int blocks_per_img, size_t npix2, float2 *__restrict__ grid) {
  const int img = blockIdx.x / blocks_per_img;
  const int u = (blockIdx.x % blocks_per_img) * kThreads + threadIdx.x;
  if (u >= n_cells) return;
  const float2 *v = vis + (size_t)img * nbc * P;
  float2 acc = make_float2(0.f, 0.f);
  const int e = off[u + 1];
  for (int q = off[u]; q < e; ++q) {
    const int bc = contrib[q];
    float2 vi;
    if (P == 2) {
      const float4 x = *reinterpret_cast<const float4 *>(v + 2 * (size_t)bc);
      vi = make_float2((x.x + x.z) * 0.5f, (x.y + x.w) * 0.5f);
    } else {
      vi = v[bc];
    }
    acc.x += vi.x;
    acc.y += vi.y;
  }
  grid[(size_t)img * npix2 + ucell[u]] = acc;
}

}  // namespace

rf_status launch_zero_f32(float *p, size_t nfloat, hipStream_t s) {
  // nfloat is a multiple of 4 for every caller (N >= 64)
  const size_t n4 = nfloat / 4;
  const int blocks = (int)std::min<size_t>((n4 + kThreads - 1) / kThreads, 8192);
  if (blocks == 0) return RF_OK;
  k_fill_zero<<<blocks, kThreads, 0, s>>>((float4 *)p, n4);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

rf_status launch_grid_dense(const rf_plan *p, const float2 *vis, int nimg, float2 *grid,
                            hipStream_t s) {
  const size_t npix2 = (size_t)p->npix * p->npix;
  rf_status st = launch_zero_f32((float *)grid, 2 * npix2 * nimg, s);
  if (st != RF_OK) return st;
  if (p->n_cells == 0 || nimg == 0) return RF_OK;
  const int bpi = (p->n_cells + kThreads - 1) / kThreads;
  const int nbc = p->nbl * p->nchan;
  const size_t blocks = (size_t)bpi * nimg;
  if (p->npol == 2)
    k_grid_cells<2><<<(unsigned)blocks, kThreads, 0, s>>>(vis, nbc, p->d_ucell, p->d_ucell_off,
                                                          p->d_contrib, p->n_cells, bpi, npix2,
                                                          grid);
  else
    k_grid_cells<1><<<(unsigned)blocks, kThreads, 0, s>>>(vis, nbc, p->d_ucell, p->d_ucell_off,
                                                          p->d_contrib, p->n_cells, bpi, npix2,
                                                          grid);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}
