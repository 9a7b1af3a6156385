// C ABI of librf: argument checking, plan construction and dispatch.
//
// Every entry point validates all of its arguments on the host before
// anything is enqueued, so an error status means the stream was not touched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "rf_internal.h"

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
bool finite(double x) { return std::isfinite(x); }

struct TableLayout {
  size_t freq, uvw, dm, delay, cells, contrib, ucell, ucell_off, rows, row_slot, tw;
  size_t rp_row, rp_sa, rp_sb, zs_off, zs_u, zs_ck, zs_cmk, cblk, total;
};

TableLayout table_layout(const rf_plan_desc *d) {
  TableLayout L{};
  const size_t bc = (size_t)d->nbl * d->nchan;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.freq = take(sizeof(double) * d->nchan);
  L.uvw = take(sizeof(double) * 3 * d->nbl);
  L.dm = take(sizeof(double) * d->ndm);
  L.delay = take(sizeof(int32_t) * (size_t)d->ndm * d->nchan);
  L.cells = take(sizeof(int32_t) * 2 * bc);
  L.contrib = take(sizeof(int32_t) * bc);
  L.ucell = take(sizeof(int32_t) * bc);
  L.ucell_off = take(sizeof(int32_t) * (bc + 1));
  L.rows = take(sizeof(int32_t) * d->npix);
  L.row_slot = take(sizeof(int32_t) * d->npix);
  L.tw = take(sizeof(float2) * d->npix);
  L.rp_row = take(sizeof(int32_t) * d->npix);
  L.rp_sa = take(sizeof(int32_t) * d->npix);
  L.rp_sb = take(sizeof(int32_t) * d->npix);
  L.zs_off = take(sizeof(int32_t) * (d->npix + 1));
  L.zs_u = take(sizeof(int32_t) * 2 * bc);
  L.zs_ck = take(sizeof(int32_t) * 2 * bc);
  L.zs_cmk = take(sizeof(int32_t) * 2 * bc);
  L.cblk = take(sizeof(int4) * (bc + 1));
  L.total = o;
  return L;
}

rf_status validate_desc(const rf_plan_desc *d) {
  if (!d) return RF_EINVAL;
  if (d->nint < 1 || d->nbl < 1 || d->nchan < 1) return RF_ESHAPE;
  if (d->npol != 1 && d->npol != 2) return RF_ESHAPE;
  if (d->vis_dtype != RF_CF32 && d->vis_dtype != RF_CF16) return RF_EINVAL;
  if (d->nbl > 65535 || d->nchan > (1 << 20)) return RF_ERANGE;
  if ((int64_t)d->nbl * d->nchan * d->npol >= (int64_t)1 << 30) return RF_ERANGE;
  if ((int64_t)d->nint * d->nbl * d->nchan * d->npol >= (int64_t)1 << 40) return RF_ERANGE;
  if (!d->freq_ghz || !d->uvw_m || !d->dm || !d->width) return RF_EINVAL;
  if (d->ndm < 1 || d->ndm > 65535 || d->nwidth < 1 || d->nwidth > 64) return RF_ESHAPE;
  if (!(d->tint_s > 0.0) || !finite(d->tint_s)) return RF_ERANGE;
  if (!(d->kdm >= 0.0) || !finite(d->kdm)) return RF_ERANGE;
  if (!(d->du > 0.0) || !finite(d->du) || !(d->dv > 0.0) || !finite(d->dv)) return RF_ERANGE;
  if (!std::isfinite(d->threshold)) return RF_ERANGE;
  if (!is_pow2(d->npix) || d->npix < 64 || d->npix > 2048) return RF_ERANGE;
  if (d->t_begin < 0 || d->t_end < d->t_begin || d->t_end > d->nint) return RF_ERANGE;
  double fmin = 1e300, fmax = 0.0;
  for (int c = 0; c < d->nchan; ++c) {
    const double f = d->freq_ghz[c];
    if (!(f > 0.0) || !finite(f)) return RF_ERANGE;
    fmin = std::min(fmin, f);
    fmax = std::max(fmax, f);
  }
  for (int i = 0; i < 3 * d->nbl; ++i)
    if (!finite(d->uvw_m[i])) return RF_ERANGE;
  double dmax = 0.0;
  for (int i = 0; i < d->ndm; ++i) {
    if (!(d->dm[i] >= 0.0) || !finite(d->dm[i])) return RF_ERANGE;
    dmax = std::max(dmax, d->dm[i]);
  }
  for (int j = 0; j < d->nwidth; ++j)
    if (d->width[j] < 1 || d->width[j] > d->nint) return RF_ERANGE;
  // the largest delay must fit comfortably in int32 (bound only; the table
  // itself is computed on the device)
  const double bound = d->kdm * dmax * (1.0 / (fmin * fmin)) / d->tint_s;
  if (!(bound < 1.0e9)) return RF_ERANGE;
  // uv cells must fit in int32 as well
  double umax = 0.0;
  for (int b = 0; b < d->nbl; ++b)
    umax = std::max({umax, std::fabs(d->uvw_m[3 * b]), std::fabs(d->uvw_m[3 * b + 1])});
  const double cmax = umax * fmax * 1e9 / 299792458.0 / std::min(d->du, d->dv);
  if (!(cmax < 1.0e9)) return RF_ERANGE;
  return RF_OK;
}

// exp(+2 pi i m / N) from float64 with exact quadrant symmetry.
float2 unit_root(int m, int N) {
  m &= N - 1;
  const int q4 = N / 4;
  const int q = m / q4, r = m % q4;
  const double two_pi = 6.283185307179586476925286766559;
  double c, s;
  if (2 * r <= q4) {
    const double a = two_pi * r / N;
    c = std::cos(a);
    s = std::sin(a);
  } else {
    const double a = two_pi * (q4 - r) / N;
    c = std::sin(a);
    s = std::cos(a);
  }
  for (int i = 0; i < q; ++i) {
    const double t = c;
    c = -s;
    s = t;
  }
  return make_float2((float)c, (float)s);
}

rf_status build_plan(const rf_plan_desc *d, void *d_tables, hipStream_t s, rf_plan *p) {
  const TableLayout L = table_layout(d);
  char *base = static_cast<char *>(d_tables);
  const int N = d->npix;
  const size_t nbc = (size_t)d->nbl * d->nchan;

  p->nint = d->nint;
  p->nbl = d->nbl;
  p->nchan = d->nchan;
  p->npol = d->npol;
  p->vis_dtype = d->vis_dtype;
  p->ndm = d->ndm;
  p->nwidth = d->nwidth;
  p->npix = N;
  // default batch budget: 240 MB keeps the two lanes' row-transformed batches
  // in the 256 MB last-level cache at 1024^2 and below; 2048^2 batches hold
  // only a few image pairs at that size, and more pairs per batch pay more
  // than the cache residency (measured: 1920 MB, 8% faster per DM trial)
  p->m_budget_mb = N >= 2048 ? 1920 : 240;
  p->tint_s = d->tint_s;
  p->du = d->du;
  p->dv = d->dv;
  p->kdm = d->kdm;
  p->threshold = d->threshold;
  p->t_begin = d->t_begin;
  p->t_end = d->t_end;
  p->freq.assign(d->freq_ghz, d->freq_ghz + d->nchan);
  p->uvw.assign(d->uvw_m, d->uvw_m + 3 * d->nbl);
  p->dm.assign(d->dm, d->dm + d->ndm);
  p->width.assign(d->width, d->width + d->nwidth);

  double *d_freq = (double *)(base + L.freq);
  double *d_uvw = (double *)(base + L.uvw);
  double *d_dm = (double *)(base + L.dm);
  p->d_delay = (int32_t *)(base + L.delay);
  p->d_cells = (int32_t *)(base + L.cells);
  p->d_contrib = (int32_t *)(base + L.contrib);
  p->d_ucell = (int32_t *)(base + L.ucell);
  p->d_ucell_off = (int32_t *)(base + L.ucell_off);
  p->d_rows = (int32_t *)(base + L.rows);
  p->d_row_slot = (int32_t *)(base + L.row_slot);
  p->d_tw = (float2 *)(base + L.tw);
  p->d_rp_row = (int32_t *)(base + L.rp_row);
  p->d_rp_sa = (int32_t *)(base + L.rp_sa);
  p->d_rp_sb = (int32_t *)(base + L.rp_sb);
  p->d_zs_off = (int32_t *)(base + L.zs_off);
  p->d_zs_u = (int32_t *)(base + L.zs_u);
  p->d_zs_ck = (int32_t *)(base + L.zs_ck);
  p->d_zs_cmk = (int32_t *)(base + L.zs_cmk);
  p->d_cblk = (int4 *)(base + L.cblk);
  p->d_freq = d_freq;
  p->d_uvw = d_uvw;

  RF_HIP_TRY(hipMemcpyAsync(d_freq, p->freq.data(), sizeof(double) * d->nchan,
                            hipMemcpyHostToDevice, s));
  RF_HIP_TRY(hipMemcpyAsync(d_uvw, p->uvw.data(), sizeof(double) * 3 * d->nbl,
                            hipMemcpyHostToDevice, s));
  RF_HIP_TRY(hipMemcpyAsync(d_dm, p->dm.data(), sizeof(double) * d->ndm, hipMemcpyHostToDevice,
                            s));
  const double nu_ref = *std::max_element(p->freq.begin(), p->freq.end());
  rf_status st = launch_plan_tables(d_freq, d_uvw, d_dm, d->nchan, d->nbl, d->ndm, nu_ref,
                                    d->tint_s, d->kdm, d->du, d->dv, p->d_delay, p->d_cells, s);
  if (st != RF_OK) return st;
  p->h_delay.resize((size_t)d->ndm * d->nchan);
  p->h_cells.resize(2 * nbc);
  RF_HIP_TRY(hipMemcpyAsync(p->h_delay.data(), p->d_delay, sizeof(int32_t) * p->h_delay.size(),
                            hipMemcpyDeviceToHost, s));
  RF_HIP_TRY(hipMemcpyAsync(p->h_cells.data(), p->d_cells, sizeof(int32_t) * p->h_cells.size(),
                            hipMemcpyDeviceToHost, s));
  RF_HIP_TRY(hipStreamSynchronize(s));

  // cell-sorted contributor order
  const int lim = N / 2 - 1;
  std::vector<std::pair<int32_t, int32_t>> kv;
  kv.reserve(nbc);
  for (size_t bc = 0; bc < nbc; ++bc) {
    const int iu = p->h_cells[2 * bc], iv = p->h_cells[2 * bc + 1];
    if (iu < -lim || iu > lim || iv < -lim || iv > lim) continue;
    const int row = ((iv % N) + N) % N, col = ((iu % N) + N) % N;
    kv.emplace_back(row * N + col, (int32_t)bc);
  }
  std::sort(kv.begin(), kv.end());
  p->W = (int32_t)kv.size();
  p->n_dropped = (int32_t)(nbc - kv.size());
  std::vector<int32_t> contrib(kv.size()), ucell, off;
  std::vector<char> occ(N, 0);
  for (size_t q = 0; q < kv.size(); ++q) {
    contrib[q] = kv[q].second;
    if (q == 0 || kv[q].first != kv[q - 1].first) {
      ucell.push_back(kv[q].first);
      off.push_back((int32_t)q);
      occ[kv[q].first / N] = 1;
    }
  }
  off.push_back((int32_t)kv.size());
  p->n_cells = (int32_t)ucell.size();
  // Stored rows: the band |v| <= vmax of the Hermitian-symmetrised grid in
  // row order v = -vmax .. vmax, so that a row's slot is (r + vmax) mod N;
  // empty rows inside the band are transformed as zeros.
  int vmax = -1;
  for (int r = 0; r < N; ++r)
    if (occ[r]) vmax = std::max(vmax, std::min(r, N - r));
  p->vmax = vmax;
  std::vector<int32_t> rows, row_slot(N, -1);
  for (int v = -vmax; v <= vmax; ++v) {
    const int r = v & (N - 1);
    row_slot[r] = (int32_t)rows.size();  // = band_slot(r, N, vmax)
    rows.push_back(r);
  }
  p->n_rows = (int32_t)rows.size();
  std::vector<float2> tw(N);
  for (int m = 0; m < N; ++m) tw[m] = unit_root(m, N);

  // Z positions per row pair {v, -v}: the union of row v's own cells and the
  // mirrors of row -v's cells, each with both cell indices.
  std::vector<int32_t> row_begin(N + 1, 0);
  for (int32_t c = 0; c < p->n_cells; ++c) row_begin[ucell[c] / N + 1]++;
  for (int r = 0; r < N; ++r) row_begin[r + 1] += row_begin[r];
  std::vector<int32_t> rp_row, rp_sa, rp_sb, zs_off, zs_u, zs_ck, zs_cmk;
  zs_off.push_back(0);
  std::vector<std::pair<int32_t, std::pair<int32_t, int32_t>>> tmp;
  for (size_t sidx = 0; sidx < rows.size(); ++sidx) {
    const int r = rows[sidx], rm = (N - r) & (N - 1);
    if (r > N / 2) continue;  // the pair is handled from its lower row
    rp_row.push_back(r);
    rp_sa.push_back((int32_t)sidx);
    rp_sb.push_back(row_slot[rm]);
    tmp.clear();
    for (int32_t c = row_begin[r]; c < row_begin[r + 1]; ++c)
      tmp.push_back({ucell[c] % N, {c, -1}});
    for (int32_t c = row_begin[rm]; c < row_begin[rm + 1]; ++c)
      tmp.push_back({(N - ucell[c] % N) & (N - 1), {-1, c}});
    std::sort(tmp.begin(), tmp.end());
    for (size_t q = 0; q < tmp.size();) {
      int32_t u = tmp[q].first, ck = -1, cmk = -1;
      while (q < tmp.size() && tmp[q].first == u) {
        if (tmp[q].second.first >= 0) ck = tmp[q].second.first;
        if (tmp[q].second.second >= 0) cmk = tmp[q].second.second;
        ++q;
      }
      zs_u.push_back(u);
      zs_ck.push_back(ck);
      zs_cmk.push_back(cmk);
    }
    zs_off.push_back((int32_t)zs_u.size());
  }
  p->n_rp = (int32_t)rp_row.size();
  // cell blocks of at most kCellBlock contributors for the staged gather
  std::vector<int32_t> cblk;
  for (int32_t c = 0; c < p->n_cells;) {
    cblk.push_back(c);
    int32_t e = c + 1;
    while (e < p->n_cells && off[e + 1] - off[c] <= kCellBlock && e - c < kCellBlock) ++e;
    c = e;
  }
  cblk.push_back(p->n_cells);
  p->n_cblk = (int32_t)cblk.size() - 1;
  p->n_zs = (int32_t)zs_u.size();

  if (!contrib.empty())
    RF_HIP_TRY(hipMemcpyAsync(p->d_contrib, contrib.data(), sizeof(int32_t) * contrib.size(),
                              hipMemcpyHostToDevice, s));
  if (!ucell.empty())
    RF_HIP_TRY(hipMemcpyAsync(p->d_ucell, ucell.data(), sizeof(int32_t) * ucell.size(),
                              hipMemcpyHostToDevice, s));
  RF_HIP_TRY(hipMemcpyAsync(p->d_ucell_off, off.data(), sizeof(int32_t) * off.size(),
                            hipMemcpyHostToDevice, s));
  if (!rows.empty())
    RF_HIP_TRY(hipMemcpyAsync(p->d_rows, rows.data(), sizeof(int32_t) * rows.size(),
                              hipMemcpyHostToDevice, s));
  RF_HIP_TRY(hipMemcpyAsync(p->d_row_slot, row_slot.data(), sizeof(int32_t) * N,
                            hipMemcpyHostToDevice, s));
  RF_HIP_TRY(hipMemcpyAsync(p->d_tw, tw.data(), sizeof(float2) * N, hipMemcpyHostToDevice, s));
  RF_HIP_TRY(hipMemcpyAsync(p->d_zs_off, zs_off.data(), sizeof(int32_t) * zs_off.size(),
                            hipMemcpyHostToDevice, s));
  if (p->n_rp > 0) {
    const size_t rb = sizeof(int32_t) * p->n_rp;
    RF_HIP_TRY(hipMemcpyAsync(p->d_rp_row, rp_row.data(), rb, hipMemcpyHostToDevice, s));
    RF_HIP_TRY(hipMemcpyAsync(p->d_rp_sa, rp_sa.data(), rb, hipMemcpyHostToDevice, s));
    RF_HIP_TRY(hipMemcpyAsync(p->d_rp_sb, rp_sb.data(), rb, hipMemcpyHostToDevice, s));
  }
  // per block: its cells and its run of contributors, in one 16-byte entry
  std::vector<int4> cblk4(p->n_cblk);
  for (int32_t b = 0; b < p->n_cblk; ++b)
    cblk4[b] = make_int4(cblk[b], cblk[b + 1], off[cblk[b]], off[cblk[b + 1]]);
  if (p->n_cblk > 0)
    RF_HIP_TRY(hipMemcpyAsync(p->d_cblk, cblk4.data(), sizeof(int4) * cblk4.size(),
                              hipMemcpyHostToDevice, s));
  if (p->n_zs > 0) {
    const size_t zb = sizeof(int32_t) * p->n_zs;
    RF_HIP_TRY(hipMemcpyAsync(p->d_zs_u, zs_u.data(), zb, hipMemcpyHostToDevice, s));
    RF_HIP_TRY(hipMemcpyAsync(p->d_zs_ck, zs_ck.data(), zb, hipMemcpyHostToDevice, s));
    RF_HIP_TRY(hipMemcpyAsync(p->d_zs_cmk, zs_cmk.data(), zb, hipMemcpyHostToDevice, s));
  }
  RF_HIP_TRY(hipStreamSynchronize(s));

  p->max_delay = p->h_delay.empty() ? 0 : *std::max_element(p->h_delay.begin(), p->h_delay.end());
  p->n_images = 0;
  p->img_base.assign((size_t)d->ndm * d->nwidth, 0);
  int64_t per_dm = 0;
  for (int j = 0; j < d->nwidth; ++j) per_dm += d->nint / d->width[j];
  for (int i = 0; i < d->ndm; ++i) {
    int64_t b = (int64_t)i * per_dm;
    for (int j = 0; j < d->nwidth; ++j) {
      p->img_base[(size_t)i * d->nwidth + j] = b;
      b += d->nint / d->width[j];
    }
  }
  p->n_images = per_dm * d->ndm;
  p->table_bytes = L.total;
  return RF_OK;
}

size_t vis_elem_bytes(const rf_plan *p) { return (size_t)p->npol * (p->vis_dtype == RF_CF32 ? 8 : 4); }

}  // namespace

extern "C" {

const char *rf_status_string(rf_status s) {
  switch (s) {
    case RF_OK: return "ok";
    case RF_EINVAL: return "invalid argument";
    case RF_ESHAPE: return "shape mismatch";
    case RF_ERANGE: return "value out of range";
    case RF_EWORKSPACE: return "workspace or table buffer too small";
    case RF_EHIP: return "HIP runtime error";
    case RF_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

rf_status rf_plan_table_bytes(const rf_plan_desc *desc, size_t *bytes) {
  if (!bytes) return RF_EINVAL;
  const rf_status st = validate_desc(desc);
  if (st != RF_OK) return st;
  *bytes = table_layout(desc).total;
  return RF_OK;
}

rf_status rf_plan_create(const rf_plan_desc *desc, void *d_tables, size_t bytes, void *stream,
                         rf_plan **out) {
  if (!out) return RF_EINVAL;
  *out = nullptr;
  const rf_status st = validate_desc(desc);
  if (st != RF_OK) return st;
  if (!d_tables) return RF_EINVAL;
  if (bytes < table_layout(desc).total) return RF_EWORKSPACE;
  rf_plan *p = new (std::nothrow) rf_plan();
  if (!p) return RF_EHIP;
  const rf_status bs = build_plan(desc, d_tables, (hipStream_t)stream, p);
  if (bs != RF_OK) {
    delete p;
    return bs;
  }
  *out = p;
  return RF_OK;
}

rf_status rf_plan_destroy(rf_plan *plan) {
  delete plan;
  return RF_OK;
}

rf_status rf_plan_query(const rf_plan *p, rf_plan_info *info) {
  if (!p || !info) return RF_EINVAL;
  info->n_images = p->n_images;
  info->n_valid = p->W;
  info->n_dropped = p->n_dropped;
  info->n_cells = p->n_cells;
  info->n_rows = p->n_rows;
  info->max_delay = p->max_delay;
  info->npix = p->npix;
  info->table_bytes = p->table_bytes;
  info->lanes = p->lanes;
  info->m_budget_mb = p->m_budget_mb;
  return RF_OK;
}

rf_status rf_subtract_mean(const rf_plan *p, void *d_vis, void *stream) {
  if (!p || !d_vis) return RF_EINVAL;
  return launch_mean_subtract(p, d_vis, (hipStream_t)stream);
}

rf_status rf_noise(const rf_plan *p, uint64_t seed, uint32_t stream, int64_t t_first, void *d_vis,
                   void *stream_) {
  if (!p || !d_vis) return RF_EINVAL;
  const int64_t per = (int64_t)p->nbl * p->nchan * p->npol;
  if (t_first < 0 || (per > 0 && t_first > (INT64_MAX / 4) / per - p->nint)) return RF_ERANGE;
  return launch_noise(p, seed, stream, t_first, d_vis, (hipStream_t)stream_);
}

rf_status rf_inject(const rf_plan *p, const rf_mock *h_mocks, int32_t nmock, int64_t t_first,
                    void *d_vis, void *stream) {
  if (!p || !d_vis || nmock < 0 || (nmock > 0 && !h_mocks)) return RF_EINVAL;
  if (t_first < 0 || t_first > ((int64_t)1 << 50)) return RF_ERANGE;
  for (int k = 0; k < nmock; ++k) {
    const rf_mock &m = h_mocks[k];
    const double v[6] = {m.dm, m.t0, m.width, m.l, m.m, m.amp};
    for (double x : v)
      if (!std::isfinite(x)) return RF_ERANGE;
    if (!(m.width > 0.0) || std::fabs(m.t0) > 1e15 || std::fabs(m.dm) > 1e9) return RF_ERANGE;
  }
  return launch_inject(p, h_mocks, nmock, t_first, d_vis, (hipStream_t)stream);
}

static bool periodic_shape_ok(const rf_plan *p) {
  return p->nint >= 2 && p->nint <= 8192 && (p->nint & (p->nint - 1)) == 0;
}

rf_status rf_periodic_workspace_bytes(const rf_plan *p, size_t *bytes) {
  if (!p || !bytes) return RF_EINVAL;
  if (!periodic_shape_ok(p)) return RF_ERANGE;
  *bytes = periodic_ws_bytes(p);
  return RF_OK;
}

rf_status rf_search_periodic(const rf_plan *p, const void *d_vis, rf_candidate *d_cand,
                             int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats, void *d_ws,
                             size_t ws_bytes, void *stream) {
  if (!p || !d_vis || !d_ncand || !d_ws || (cap > 0 && !d_cand)) return RF_EINVAL;
  if (cap < 0 || !periodic_shape_ok(p)) return RF_ERANGE;
  if (ws_bytes < periodic_ws_bytes(p)) return RF_EWORKSPACE;
  return run_periodic(p, d_vis, d_cand, cap, d_ncand, d_stats, d_ws, (hipStream_t)stream);
}

rf_status rf_products_workspace_bytes(const rf_plan *p, int32_t nspec, size_t *bytes) {
  if (!p || !bytes) return RF_EINVAL;
  if (nspec < 1 || nspec > 4096) return RF_ERANGE;
  *bytes = products_ws_bytes(p, nspec);
  return RF_OK;
}

rf_status rf_candidate_products(const rf_plan *p, const void *d_vis, const rf_candidate *h_cand,
                                int32_t ncand, int32_t half, int32_t nspec, float *d_cutout,
                                float *d_spec, void *d_ws, size_t ws_bytes, void *stream) {
  if (!p || !d_vis || ncand < 0 || (ncand > 0 && !h_cand)) return RF_EINVAL;
  if (nspec < 1 || nspec > 4096 || half < 1 || half > p->npix / 2) return RF_ERANGE;
  for (int n = 0; n < ncand; ++n) {
    const rf_candidate &c = h_cand[n];
    if (c.dm_idx < 0 || c.dm_idx >= p->ndm || c.width_idx < 0 || c.width_idx >= p->nwidth)
      return RF_ERANGE;
    const int w = p->width[c.width_idx];
    if (c.t_int < 0 || c.t_int % w != 0 || c.t_int / w >= p->nint / w) return RF_ERANGE;
    if (c.x < 0 || c.x >= p->npix || c.y < 0 || c.y >= p->npix) return RF_ERANGE;
  }
  if (ncand == 0 || (!d_cutout && !d_spec)) return RF_OK;
  if (!d_ws) return RF_EINVAL;
  if (ws_bytes < products_ws_bytes(p, nspec)) return RF_EWORKSPACE;
  return run_products(p, d_vis, h_cand, ncand, half, nspec, d_cutout, d_spec, d_ws,
                      (hipStream_t)stream);
}

rf_status rf_select_tier(const rf_candidate *h_in, int32_t n, float threshold,
                         rf_candidate *h_out, int32_t cap, int32_t *nout) {
  if (!nout || (n > 0 && !h_in) || (cap > 0 && !h_out)) return RF_EINVAL;
  if (n < 0 || cap < 0 || !std::isfinite(threshold)) return RF_ERANGE;
  int32_t k = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (h_in[i].snr > threshold) {
      if (k < cap) h_out[k] = h_in[i];  // k <= i: in place is safe
      ++k;
    }
  }
  *nout = k;
  return RF_OK;
}

rf_status rf_plan_set_tuning(rf_plan *p, int32_t lanes, int32_t m_budget_mb) {
  if (!p) return RF_EINVAL;
  if (lanes < 1 || lanes > 4 || m_budget_mb < 16 || m_budget_mb > 4096) return RF_ERANGE;
  p->lanes = lanes;
  p->m_budget_mb = m_budget_mb;
  return RF_OK;
}

rf_status rf_batch_workspace_bytes(const rf_plan *const *plans, int32_t nseg, size_t *bytes) {
  if (!plans || !bytes || nseg < 1) return RF_EINVAL;
  for (int i = 0; i < nseg; ++i)
    if (!plans[i]) return RF_EINVAL;
  *bytes = batch_ws_bytes(plans, nseg, nullptr);
  return RF_OK;
}

rf_status rf_batch_create(const rf_plan *const *plans, int32_t nseg, const void *const *d_vis,
                          rf_candidate *const *d_cand, const int32_t *cap,
                          int32_t *const *d_ncand, rf_image_stats *const *d_stats, void *d_ws,
                          size_t ws_bytes, int32_t flags, rf_batch **out) {
  if (!out) return RF_EINVAL;
  *out = nullptr;
  if (!plans || nseg < 1 || !d_vis || !d_cand || !cap || !d_ncand || !d_ws) return RF_EINVAL;
  if (flags & ~RF_BATCH_GRAPH) return RF_EINVAL;
  for (int i = 0; i < nseg; ++i) {
    if (!plans[i] || !d_vis[i] || !d_ncand[i]) return RF_EINVAL;
    if (cap[i] < 0) return RF_ERANGE;
    if (cap[i] > 0 && !d_cand[i]) return RF_EINVAL;
  }
  return batch_create(plans, nseg, d_vis, d_cand, cap, d_ncand, d_stats, d_ws, ws_bytes, flags,
                      out);
}

rf_status rf_batch_graph_nodes(const rf_batch *b, size_t *nodes) {
  if (!b || !nodes) return RF_EINVAL;
  *nodes = batch_graph_nodes(b);
  return RF_OK;
}

rf_status rf_batch_run(rf_batch *b, void *stream) {
  if (!b) return RF_EINVAL;
  return batch_run(b, (hipStream_t)stream);
}

rf_status rf_batch_destroy(rf_batch *b) {
  if (!b) return RF_EINVAL;
  batch_destroy(b);
  return RF_OK;
}

rf_status rf_get_delays(const rf_plan *p, int32_t *h_out) {
  if (!p || !h_out) return RF_EINVAL;
  std::memcpy(h_out, p->h_delay.data(), sizeof(int32_t) * p->h_delay.size());
  return RF_OK;
}

rf_status rf_get_cells(const rf_plan *p, int32_t *h_out) {
  if (!p || !h_out) return RF_EINVAL;
  std::memcpy(h_out, p->h_cells.data(), sizeof(int32_t) * p->h_cells.size());
  return RF_OK;
}

rf_status rf_workspace_bytes(const rf_plan *p, int32_t op, int64_t nimg, size_t *bytes) {
  if (!p || !bytes) return RF_EINVAL;
  switch (op) {
    case RF_OP_IMAGE:
      if (nimg < 0) return RF_ERANGE;
      *bytes = image_ws_bytes(p, nimg);
      return RF_OK;
    case RF_OP_SEARCH:
      if (nimg < 0) return RF_ERANGE;
      *bytes = 0;
      return RF_OK;
    case RF_OP_SEGMENT:
      *bytes = segment_ws_bytes(p);
      return RF_OK;
    case RF_OP_SEGMENT_STEPS:
      *bytes = steps_ws_bytes(p);
      return RF_OK;
    default:
      return RF_EINVAL;
  }
}

rf_status rf_dedisperse(const rf_plan *p, int32_t dm_idx, const void *d_vis, void *d_out,
                        void *stream) {
  if (!p || !d_vis || !d_out) return RF_EINVAL;
  if (dm_idx < 0 || dm_idx >= p->ndm) return RF_ERANGE;
  const size_t bytes = (size_t)p->nint * p->nbl * p->nchan * vis_elem_bytes(p);
  const char *a = (const char *)d_vis, *b = (const char *)d_out;
  if (a < b + bytes && b < a + bytes) return RF_EINVAL;  // must not overlap
  return launch_dedisperse(p, p->d_delay + (size_t)dm_idx * p->nchan, d_vis, d_out,
                           (hipStream_t)stream);
}

rf_status rf_resample(const rf_plan *p, int32_t width, const void *d_in, int32_t nin,
                      void *d_out, void *stream) {
  if (!p) return RF_EINVAL;
  if (width < 1 || nin < 0) return RF_ERANGE;
  if (nin / width == 0) return RF_OK;
  if (!d_in || !d_out) return RF_EINVAL;
  return launch_resample(p, width, d_in, p->vis_dtype, nin, (float2 *)d_out,
                         (hipStream_t)stream);
}

rf_status rf_grid(const rf_plan *p, const void *d_vis, int32_t nimg, void *d_grid,
                  void *stream) {
  if (!p) return RF_EINVAL;
  if (nimg < 0) return RF_ERANGE;
  if (nimg == 0) return RF_OK;
  if (!d_vis || !d_grid) return RF_EINVAL;
  return launch_grid_dense(p, (const float2 *)d_vis, nimg, (float2 *)d_grid,
                           (hipStream_t)stream);
}

rf_status rf_image(const rf_plan *p, const void *d_grid, int32_t nimg, float *d_img, void *d_ws,
                   size_t ws_bytes, void *stream) {
  if (!p) return RF_EINVAL;
  if (nimg < 0) return RF_ERANGE;
  if (nimg == 0) return RF_OK;
  if (!d_grid || !d_img) return RF_EINVAL;
  const size_t need = image_ws_bytes(p, nimg);
  if (ws_bytes < need) return RF_EWORKSPACE;
  if (need > 0 && !d_ws) return RF_EINVAL;
  return launch_image_dense(p, (const float2 *)d_grid, nimg, d_img, (float2 *)d_ws,
                            (hipStream_t)stream);
}

rf_status rf_search(const rf_plan *p, const float *d_img, int32_t nimg, const rf_image_tag *d_tags,
                    rf_image_stats *d_stats, rf_candidate *d_cand, int32_t cap, int32_t *d_ncand,
                    void *d_ws, size_t ws_bytes, void *stream) {
  (void)d_ws;
  (void)ws_bytes;
  if (!p) return RF_EINVAL;
  if (nimg < 0 || cap < 0) return RF_ERANGE;
  if (nimg == 0) return RF_OK;
  if (!d_img || !d_tags || !d_ncand || (cap > 0 && !d_cand)) return RF_EINVAL;
  return launch_search(p, d_img, nimg, d_tags, nullptr, d_stats, d_cand, cap, d_ncand,
                       (hipStream_t)stream);
}

rf_status rf_search_segment(const rf_plan *p, const void *d_vis, rf_candidate *d_cand,
                            int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats, void *d_ws,
                            size_t ws_bytes, void *stream) {
  if (!p) return RF_EINVAL;
  if (cap < 0) return RF_ERANGE;
  if (!d_vis || !d_ncand || (cap > 0 && !d_cand)) return RF_EINVAL;
  const size_t need = segment_ws_bytes(p);
  if (ws_bytes < need) return RF_EWORKSPACE;
  if (!d_ws) return RF_EINVAL;
  return run_segment(p, d_vis, d_cand, cap, d_ncand, d_stats, d_ws, ws_bytes,
                     (hipStream_t)stream, nullptr);
}

rf_status rf_search_segment_begin(const rf_plan *p, const void *d_vis, rf_candidate *d_cand,
                                  int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats,
                                  void *d_ws, size_t ws_bytes, void *stream,
                                  rf_segment_job **job) {
  if (!job) return RF_EINVAL;
  *job = nullptr;
  if (!p) return RF_EINVAL;
  if (cap < 0) return RF_ERANGE;
  if (!d_vis || !d_ncand || (cap > 0 && !d_cand)) return RF_EINVAL;
  if (ws_bytes < segment_ws_bytes(p)) return RF_EWORKSPACE;
  if (!d_ws) return RF_EINVAL;
  return segment_begin(p, d_vis, d_cand, cap, d_ncand, d_stats, d_ws, ws_bytes,
                       (hipStream_t)stream, job);
}

rf_status rf_search_segment_end(rf_segment_job *job) {
  if (!job) return RF_EINVAL;
  return segment_end(job);
}

rf_status rf_search_segment_profile(const rf_plan *p, const void *d_vis, rf_candidate *d_cand,
                                    int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats,
                                    void *d_ws, size_t ws_bytes, void *stream,
                                    rf_kernel_times *times) {
  if (!p || !times) return RF_EINVAL;
  if (cap < 0) return RF_ERANGE;
  if (!d_vis || !d_ncand || (cap > 0 && !d_cand)) return RF_EINVAL;
  const size_t need = segment_ws_bytes(p);
  if (ws_bytes < need) return RF_EWORKSPACE;
  if (!d_ws) return RF_EINVAL;
  if (times->concurrent != 0 && times->concurrent != 1) return RF_EINVAL;
  if (times->sample < 0) return RF_ERANGE;
  const int32_t conc = times->concurrent, smp = times->sample;
  std::memset(times, 0, sizeof(*times));
  times->concurrent = conc;
  times->sample = smp;
  return run_segment(p, d_vis, d_cand, cap, d_ncand, d_stats, d_ws, ws_bytes,
                     (hipStream_t)stream, times);
}

rf_status rf_search_segment_steps(const rf_plan *p, const void *d_vis, rf_candidate *d_cand,
                                  int32_t cap, int32_t *d_ncand, rf_image_stats *d_stats,
                                  void *d_ws, size_t ws_bytes, void *stream) {
  if (!p) return RF_EINVAL;
  if (cap < 0) return RF_ERANGE;
  if (!d_vis || !d_ncand || (cap > 0 && !d_cand)) return RF_EINVAL;
  const size_t need = steps_ws_bytes(p);
  if (ws_bytes < need) return RF_EWORKSPACE;
  if (!d_ws) return RF_EINVAL;
  return run_segment_steps(p, d_vis, d_cand, cap, d_ncand, d_stats, d_ws, ws_bytes,
                           (hipStream_t)stream);
}

}  // extern "C"
