// 2-D FFT imaging (Law et al. 2018, section 3.2: "the 2d FFT for imaging").
//
//   img[Y][X] = (1/W) Re sum_{iu,iv} G[iv][iu] exp(+2 pi i (iu (X - N/2) + iv (Y - N/2)) / N)
//
// Two images a, b share one complex transform.  The real part of an inverse
// DFT equals the inverse DFT of the Hermitian part H[k] = (G[k] + conj G[-k])/2,
// so Z = H_a + i H_b transforms to W (img_a + i img_b).  The shift of the
// phase centre to pixel (N/2, N/2) is the factor (-1)^(iu + iv) on the grid.
// Pass 1 (rows): for each occupied row v of the symmetrised grid, build Z[v][:]
// from rows v and -v of both grids in LDS and transform along u.  Rows with no
// samples are skipped and never stored.  Pass 2 (columns): gather a tile of
// columns of the row-transformed data (zero for skipped rows), transform along
// v and write Re / W and Im / W to the two images.
#include "rf_internal.h"
#include "fft.h"

namespace {

using namespace rf;

// DIRECT: one complex grid per transform (the complex image of a grid with no
// Hermitian symmetry, as in the periodicity search).  For the pair (G, -iG)
// zval reduces exactly to Z = 2 sg G (the mirrored terms cancel to exact
// zeros and sg (x + x) = (2 sg) x), so the direct form gives the pair's
// values bit for bit from one grid.
template <int N, bool DIRECT = false>
__global__ __launch_bounds__(RowCfg<N>::NT) void k_rows_dense(
    const float2 *__restrict__ grid, int nimg, const int32_t *__restrict__ rows, int n_rows,
    int row_blocks, float hw, const float2 *__restrict__ tw, float2 *__restrict__ M) {
  constexpr int F = RowCfg<N>::F, NT = RowCfg<N>::NT, S = RowCfg<N>::STRIDE;
  constexpr int PS = RowFft<N>::PS;
  __shared__ float2 buf[F * S];
  const int pair = blockIdx.x / row_blocks;
  const int slot0 = (blockIdx.x % row_blocks) * F;
  const int tid = threadIdx.x;
  const size_t npix2 = (size_t)N * N;
  const float2 *Ga = grid + (size_t)(DIRECT ? pair : 2 * pair) * npix2;
  const float2 *Gb = Ga + npix2;
  const bool hasb = 2 * pair + 1 < nimg;
  for (int e = tid; e < F * N; e += NT) {
    const int f = e / N, u = e % N;
    const int slot = slot0 + f;
    float2 z = make_float2(0.f, 0.f);
    if (slot < n_rows) {
      const int r = rows[slot];
      if (DIRECT) {
        const float2 a = Ga[(size_t)r * N + u];
        const float sg2 = 2.0f * (((r + u) & 1) ? -hw : hw);
        z = make_float2(sg2 * a.x, sg2 * a.y);
      } else {
        const int rm = (N - r) & (N - 1);
        const int um = (N - u) & (N - 1);
        const float2 a = Ga[(size_t)r * N + u], am = Ga[(size_t)rm * N + um];
        float2 b = make_float2(0.f, 0.f), bm = b;
        if (hasb) {
          b = Gb[(size_t)r * N + u];
          bm = Gb[(size_t)rm * N + um];
        }
        z = zval(a, am, b, bm, ((r + u) & 1) ? -hw : hw);
      }
    }
    buf[f * S + pidx<PS>(u)] = z;
  }
  __syncthreads();
  fft_inverse<RowFft<N>, F, NT, S, true>(
      buf, tw, tid, [&](int f, int i) { return buf[f * S + pidx<PS>(i)]; },
      [&](int f, int x, float2 v) {
        const int slot = slot0 + f;
        if (slot < n_rows) M[((size_t)pair * n_rows + slot) * N + x] = v;
      });
}

// AMP: one output image per transform, the amplitude |Re + i Im| of the
// complex image (periodicity search); otherwise Re and Im are the two images
// of the pair.
template <int N, bool AMP = false>
__global__ __launch_bounds__(ColCfg<N>::NT) void k_cols_image(
    const float2 *__restrict__ M, int n_rows, int vmax, int nimg,
    const float2 *__restrict__ tw, float *__restrict__ img) {
  constexpr int COLS = ColCfg<N>::COLS, NT = ColCfg<N>::NT, S = ColCfg<N>::STRIDE;
  constexpr int CB = N / COLS;
  __shared__ float2 buf[COLS * S];
  const int pair = blockIdx.x / CB;
  const int x0 = (blockIdx.x % CB) * COLS;
  const int tid = threadIdx.x;
  // rows outside the stored band read as zero through the range check
  const auto rm = buf_rsrc(M + (size_t)pair * n_rows * N + x0, (uint32_t)n_rows * N * 8u);
  float *ia = img + (size_t)(AMP ? pair : 2 * pair) * N * N + x0;
  float *ib = ia + (size_t)N * N;
  const bool hasb = 2 * pair + 1 < nimg;
  fft_inverse<ColFft<N>, COLS, NT, S, false>(
      buf, tw, tid,
      [&](int f, int i) { return buf_load_f2(rm, (uint32_t)(band_slot_raw(i, N, vmax) * N + f) * 8u); },
      [&](int f, int y, float2 v) {
        if (AMP) {
          ia[(size_t)y * N + f] = sqrtf(v.x * v.x + v.y * v.y);
        } else {
          ia[(size_t)y * N + f] = v.x;  // 1/W is folded into Z
          if (hasb) ib[(size_t)y * N + f] = v.y;
        }
      });
}

// COMPLEX: `nimg` complex grids -> `nimg` amplitude images (one transform
// each); otherwise `nimg` grids -> `nimg` real images, two per transform.
template <int N, bool COMPLEX>
rf_status image_dense_n(const rf_plan *p, const float2 *grid, int nimg, float *img, float2 *ws,
                        hipStream_t s) {
  const int npairs = COMPLEX ? nimg : (nimg + 1) / 2;
  if (npairs == 0) return RF_OK;
  if (p->n_rows == 0 || p->W == 0) return launch_zero_f32(img, (size_t)nimg * N * N, s);
  const int rb = (p->n_rows + RowCfg<N>::F - 1) / RowCfg<N>::F;
  k_rows_dense<N, COMPLEX><<<(unsigned)((size_t)rb * npairs), RowCfg<N>::NT, 0, s>>>(
      grid, nimg, p->d_rows, p->n_rows, rb, half_inv_w(p), p->d_tw, ws);
  RF_HIP_TRY(hipGetLastError());
  constexpr int CB = N / ColCfg<N>::COLS;
  k_cols_image<N, COMPLEX><<<(unsigned)((size_t)CB * npairs), ColCfg<N>::NT, 0, s>>>(
      ws, p->n_rows, p->vmax, nimg, p->d_tw, img);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

}  // namespace

size_t image_ws_bytes(const rf_plan *p, int64_t nimg) {
  return (size_t)((nimg + 1) / 2) * (size_t)p->n_rows * (size_t)p->npix * sizeof(float2);
}

template <bool COMPLEX>
rf_status image_dense_any(const rf_plan *p, const float2 *grid, int nimg, float *img, float2 *ws,
                          hipStream_t s) {
  switch (p->npix) {
    case 64: return image_dense_n<64, COMPLEX>(p, grid, nimg, img, ws, s);
    case 128: return image_dense_n<128, COMPLEX>(p, grid, nimg, img, ws, s);
    case 256: return image_dense_n<256, COMPLEX>(p, grid, nimg, img, ws, s);
    case 512: return image_dense_n<512, COMPLEX>(p, grid, nimg, img, ws, s);
    case 1024: return image_dense_n<1024, COMPLEX>(p, grid, nimg, img, ws, s);
    case 2048: return image_dense_n<2048, COMPLEX>(p, grid, nimg, img, ws, s);
    default: return RF_EUNSUPPORTED;
  }
}

rf_status launch_image_dense(const rf_plan *p, const float2 *grid, int nimg, float *img,
                             float2 *ws, hipStream_t s) {
  return image_dense_any<false>(p, grid, nimg, img, ws, s);
}

rf_status launch_image_amplitude(const rf_plan *p, const float2 *grid, int nimg, float *amp,
                                 float2 *ws, hipStream_t s) {
  return image_dense_any<true>(p, grid, nimg, amp, ws, s);
}
