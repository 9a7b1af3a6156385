// Internal declarations shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/rf.h"

// Contributors per cell block of the staged gather (the host forms the
// blocks, the gather kernel stages one block per workgroup).
constexpr int kCellBlock = 1024;

// Host-side plan object.  Immutable after rf_plan_create.
struct rf_plan {
  // description (scalars and host copies of the arrays)
  int32_t nint, nbl, nchan, npol, vis_dtype, ndm, nwidth, npix;
  double tint_s, du, dv, kdm;
  float threshold;
  int32_t t_begin, t_end;
  std::vector<double> freq, uvw, dm;
  std::vector<int32_t> width;
  // tuning of the fused search (rf_plan_set_tuning): lane streams and the
  // budget of all lanes' row-transformed batches, MB
  int32_t lanes = 2, m_budget_mb = 240;

  // derived
  int32_t W;          // valid (baseline, channel) pairs
  int32_t n_dropped;
  int32_t n_cells;    // distinct occupied cells
  int32_t n_rows;     // stored rows: the band |v| <= vmax (2 vmax + 1 rows)
  int32_t vmax;       // largest |v| of a gridded sample (-1 if none)
  int32_t max_delay;
  int64_t n_images;
  size_t table_bytes;
  std::vector<int64_t> img_base;  // [ndm * nwidth] first image index of (dm, width)

  // device tables (inside the caller's table buffer)
  int32_t *d_delay;         // [ndm][nchan]
  int32_t *d_cells;         // [nbl][nchan][2] (iu, iv)
  int32_t *d_contrib;       // [W] pair index b*nchan + c, sorted by (cell, pair)
  int32_t *d_ucell;         // [n_cells] linear cell (iv mod N) * N + (iu mod N), ascending
  int32_t *d_ucell_off;     // [n_cells + 1] CSR offsets into d_contrib
  int32_t *d_rows;          // [n_rows] band rows in slot order: -vmax .. vmax (mod N)
  int32_t *d_row_slot;      // [N] slot of a row in d_rows, or -1 (= band_slot)
  float2 *d_tw;             // [N] exp(+2 pi i m / N)
  // Z positions of the paired Hermitian transform, grouped by row pair
  // {v, -v} (v in [0, N/2], occupied): row pair rp has rows v = rp_row[rp]
  // (compact slot rp_sa[rp]) and -v (slot rp_sb[rp]); its positions
  // zs_off[rp] .. zs_off[rp+1] are columns zs_u of row v with zs_ck the cell
  // index (into d_ucell) at (v, u) and zs_cmk the one at (-v, -u), -1 where
  // the grid is empty.  Row -v's positions are the mirrors (-u).
  int32_t n_rp, n_zs;
  // cell blocks for the staged gather: block b is cells cblk[b].x ..
  // cblk[b].y - 1, whose contributors are cblk[b].z .. cblk[b].w - 1 of
  // d_contrib, at most kCellBlock (a single heavier cell forms its own block)
  int32_t n_cblk;
  int4 *d_cblk;             // [n_cblk]
  double *d_freq;           // [nchan] channel centres, GHz
  double *d_uvw;            // [nbl][3] baseline vectors, metres
  int32_t *d_rp_row;        // [n_rp]
  int32_t *d_rp_sa;         // [n_rp]
  int32_t *d_rp_sb;         // [n_rp]
  int32_t *d_zs_off;        // [n_rp + 1]
  int32_t *d_zs_u;          // [n_zs]
  int32_t *d_zs_ck;         // [n_zs]
  int32_t *d_zs_cmk;        // [n_zs]

  // host copies used by rf_get_* and the launchers
  std::vector<int32_t> h_delay;
  std::vector<int32_t> h_cells;
};

// Factor of the paired Hermitian Z values: 1/2 from the Hermitian part and
// the image normalisation 1/W (applied once per grid value instead of once per
// pixel).  Every path that forms Z uses this value, so their images agree bit
// for bit.
inline float half_inv_w(const rf_plan *p) { return p->W > 0 ? 0.5f * (1.0f / (float)p->W) : 0.0f; }

// Slot of grid row r in the stored band |v| <= vmax, or -1 outside it.  The
// band is stored in row order -vmax .. vmax, so the slot is (r + vmax) mod N
// and slots past 2 vmax are the rows outside the band: a column load at slot
// (r + vmax) mod N falls past the end of the band exactly when r is outside.
__host__ __device__ inline int band_slot_raw(int r, int N, int vmax) { return (r + vmax) & (N - 1); }
__host__ __device__ inline int band_slot(int r, int N, int vmax) {
  const int s = band_slot_raw(r, N, vmax);
  return s <= 2 * vmax ? s : -1;
}

#define RF_HIP_TRY(expr)                      \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return RF_EHIP;     \
  } while (0)

// ---- launchers (each returns RF_OK or RF_EHIP; arguments already validated)

// plan tables (float64, no contraction)
rf_status launch_plan_tables(const double *d_freq, const double *d_uvw, const double *d_dm,
                             int nchan, int nbl, int ndm, double nu_ref, double tint_s,
                             double kdm, double du, double dv, int32_t *d_delay,
                             int32_t *d_cells, hipStream_t s);

// dedispersion / resampling
rf_status launch_dedisperse(const rf_plan *p, const int32_t *d_delay_row, const void *in,
                            void *out, hipStream_t s);
rf_status launch_resample(const rf_plan *p, int width, const void *in, int in_dtype, int nin,
                          float2 *out, hipStream_t s);

// dense gridding: vis CF32 [nimg][nbl][nchan][npol] -> grid [nimg][N][N]
rf_status launch_grid_dense(const rf_plan *p, const float2 *vis, int nimg, float2 *grid,
                            hipStream_t s);

// imaging from dense grids; ws holds [ceil(nimg/2)][n_rows][N] float2
size_t image_ws_bytes(const rf_plan *p, int64_t nimg);
rf_status launch_image_dense(const rf_plan *p, const float2 *grid, int nimg, float *img,
                             float2 *ws, hipStream_t s);
// complex images of nimg grids (no Hermitian symmetry), written as amplitudes
// [nimg][N][N]; ws holds image_ws_bytes(p, 2 * nimg)
rf_status launch_image_amplitude(const rf_plan *p, const float2 *grid, int nimg, float *amp,
                                 float2 *ws, hipStream_t s);

// statistics, threshold and candidates
struct rf_tag_gen {       // implicit tags: image n -> (dm_idx, width_idx, (k0 + n) * w)
  int32_t dm_idx, width_idx, width, k0;
};
rf_status launch_search(const rf_plan *p, const float *img, int nimg, const rf_image_tag *tags,
                        const rf_tag_gen *gen, rf_image_stats *stats, rf_candidate *cand,
                        int cap, int32_t *ncand, hipStream_t s);
rf_status launch_search_ex(const rf_plan *p, const float *img, int nimg,
                           const rf_image_tag *tags, const rf_tag_gen *gen, rf_image_stats *stats,
                           rf_candidate *cand, int cap, int32_t *ncand, float sigma_scale,
                           int t_begin, int t_end, hipStream_t s);
rf_status launch_zero_i32(int32_t *p, int n, hipStream_t s);
rf_status launch_zero_f32(float *p, size_t nfloat, hipStream_t s);

// whole segment: fused path (k_fused.hip) and the step chain (rf_segment.cpp)
size_t segment_ws_bytes(const rf_plan *p);
rf_status launch_mean_subtract(const rf_plan *p, void *vis, hipStream_t s);

size_t steps_ws_bytes(const rf_plan *p);
rf_status run_segment_steps(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                            int32_t *ncand, rf_image_stats *stats, void *ws, size_t ws_bytes,
                            hipStream_t s);
rf_status run_segment(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                      int32_t *ncand, rf_image_stats *stats, void *ws, size_t ws_bytes,
                      hipStream_t s, rf_kernel_times *kt);
rf_status segment_begin(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                        int32_t *ncand, rf_image_stats *stats, void *ws, size_t ws_bytes,
                        hipStream_t s, rf_segment_job **out);
rf_status segment_end(rf_segment_job *j);
size_t batch_ws_bytes(const rf_plan *const *plans, int nseg, size_t *main_bytes);
rf_status batch_create(const rf_plan *const *plans, int nseg, const void *const *d_vis,
                       rf_candidate *const *d_cand, const int32_t *cap, int32_t *const *d_ncand,
                       rf_image_stats *const *d_stats, void *d_ws, size_t ws_bytes, int flags,
                       rf_batch **out);
size_t batch_graph_nodes(const rf_batch *b);
rf_status batch_run(rf_batch *b, hipStream_t s);
void batch_destroy(rf_batch *b);

// synthetic data (k_mock.hip): counter-based noise and mock transients
constexpr int kMocksPerLaunch = 64;  // mocks passed by value per injection launch
rf_status launch_noise(const rf_plan *p, uint64_t seed, uint32_t stream, int64_t t_first,
                       void *vis, hipStream_t s);
rf_status launch_inject(const rf_plan *p, const rf_mock *mocks, int nmock, int64_t t_first,
                        void *vis, hipStream_t s);

// second-tier candidate products (k_products.hip)
size_t products_ws_bytes(const rf_plan *p, int nspec);
rf_status run_products(const rf_plan *p, const void *vis, const rf_candidate *cand, int ncand,
                       int half, int nspec, float *cutout, float *spec, void *ws,
                       hipStream_t s);

// periodicity search (k_periodic.hip)
size_t periodic_ws_bytes(const rf_plan *p);
rf_status run_periodic(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                       int32_t *ncand, rf_image_stats *stats, void *ws, hipStream_t s);
