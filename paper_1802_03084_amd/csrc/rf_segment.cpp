// Whole-segment search as a chain of the step kernels: the loop of Law et al.
// 2018, Figure 2 (DM trials outside, sampling times inside, every resampled
// integration imaged and thresholded), driven from the host on one stream
// with dense intermediates in the caller's workspace.  This is the plain
// reference path; the fused path in k_fused.hip gives the same results.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rf_internal.h"

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int chunk_images(const rf_plan *p) { return p->npix >= 2048 ? 32 : 64; }

struct SegLayout {
  size_t dd, rs, grid, mws, img, total;
};

SegLayout seg_layout(const rf_plan *p) {
  SegLayout L{};
  const size_t per_int = (size_t)p->nbl * p->nchan * p->npol;
  const size_t sbytes = p->vis_dtype == RF_CF32 ? 8 : 4;
  const int ic = chunk_images(p);
  const size_t np2 = (size_t)p->npix * p->npix;
  size_t o = 0;
  L.dd = o;
  o += align_up(per_int * p->nint * sbytes);
  L.rs = o;
  o += align_up(per_int * p->nint * 8);
  L.grid = o;
  o += align_up(np2 * 8 * ic);
  L.mws = o;
  o += align_up(image_ws_bytes(p, ic));
  L.img = o;
  o += align_up(np2 * 4 * ic);
  L.total = o;
  return L;
}

}  // namespace

size_t steps_ws_bytes(const rf_plan *p) { return seg_layout(p).total; }

rf_status run_segment_steps(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                            int32_t *ncand, rf_image_stats *stats, void *ws, size_t ws_bytes,
                            hipStream_t s) {
  (void)ws_bytes;
  const SegLayout L = seg_layout(p);
  char *base = static_cast<char *>(ws);
  void *dd = base + L.dd;
  float2 *rs = (float2 *)(base + L.rs);
  float2 *grid = (float2 *)(base + L.grid);
  float2 *mws = (float2 *)(base + L.mws);
  float *img = (float *)(base + L.img);
  const size_t per_int = (size_t)p->nbl * p->nchan * p->npol;
  const int ic = chunk_images(p);

  rf_status st = launch_zero_i32(ncand, 1, s);
  if (st != RF_OK) return st;
  for (int i = 0; i < p->ndm; ++i) {
    st = launch_dedisperse(p, p->d_delay + (size_t)i * p->nchan, vis, dd, s);
    if (st != RF_OK) return st;
    for (int j = 0; j < p->nwidth; ++j) {
      const int w = p->width[j];
      const int nout = p->nint / w;
      st = launch_resample(p, w, dd, p->vis_dtype, p->nint, rs, s);
      if (st != RF_OK) return st;
      for (int k0 = 0; k0 < nout; k0 += ic) {
        const int n = std::min(ic, nout - k0);
        st = launch_grid_dense(p, rs + (size_t)k0 * per_int, n, grid, s);
        if (st != RF_OK) return st;
        st = launch_image_dense(p, grid, n, img, mws, s);
        if (st != RF_OK) return st;
        const rf_tag_gen gen{i, j, w, k0};
        rf_image_stats *st_out =
            stats ? stats + p->img_base[(size_t)i * p->nwidth + j] + k0 : nullptr;
        st = launch_search(p, img, n, nullptr, &gen, st_out, cand, cap, ncand, s);
        if (st != RF_OK) return st;
      }
    }
  }
  return RF_OK;
}
