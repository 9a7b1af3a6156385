// Plan tables: integer dispersion delays and nearest uv cells, in float64.
//
// Delay (Law et al. 2018, section 2.1 footnote: tau = K DM / nu^2), relative to
// the highest channel and rounded half-even to whole integrations:
//     d[i][c] = rint(((K * DM_i) * (1/(nu_c*nu_c) - 1/(nu_ref*nu_ref))) / t_int)
// Cell (nearest-cell gridding, the reading used for the unstated gridding of
// section 3.2):
//     iu[b][c] = rint(((u_b * (nu_c * 1e9)) / c) / du), likewise iv.
// Every operation is one IEEE float64 operation in the order written; fused
// multiply-add contraction is disabled so the integers are reproducible
// bit for bit by any IEEE float64 evaluation in the same order.
#pragma clang fp contract(off)

#include "rf_internal.h"

namespace {

constexpr double kLight = 299792458.0;  // m/s

__global__ void k_delay_table(const double *__restrict__ freq, const double *__restrict__ dm,
                              int nchan, int ndm, double nu_ref, double tint_s, double kdm,
                              int32_t *__restrict__ out) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (c >= nchan || i >= ndm) return;
  const double f = freq[c];
  const double inv = 1.0 / (f * f);
  const double inv_ref = 1.0 / (nu_ref * nu_ref);
  const double lag = (kdm * dm[i]) * (inv - inv_ref);
  const double x = lag / tint_s;
  out[(size_t)i * nchan + c] = (int32_t)__builtin_rint(x);
}

__global__ void k_cell_table(const double *__restrict__ freq, const double *__restrict__ uvw,
                             int nchan, int nbl, double du, double dv,
                             int32_t *__restrict__ out) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (c >= nchan || b >= nbl) return;
  const double fhz = freq[c] * 1e9;
  const double u = uvw[3 * b + 0];
  const double v = uvw[3 * b + 1];
  const double ul = (u * fhz) / kLight;
  const double vl = (v * fhz) / kLight;
  const size_t o = 2 * ((size_t)b * nchan + c);
  out[o + 0] = (int32_t)__builtin_rint(ul / du);
  out[o + 1] = (int32_t)__builtin_rint(vl / dv);
}

}  // namespace

rf_status launch_plan_tables(const double *d_freq, const double *d_uvw, const double *d_dm,
                             int nchan, int nbl, int ndm, double nu_ref, double tint_s,
                             double kdm, double du, double dv, int32_t *d_delay,
                             int32_t *d_cells, hipStream_t s) {
  const int nt = 256;
  dim3 g1((nchan + nt - 1) / nt, ndm);
  k_delay_table<<<g1, nt, 0, s>>>(d_freq, d_dm, nchan, ndm, nu_ref, tint_s, kdm, d_delay);
  RF_HIP_TRY(hipGetLastError());
  dim3 g2((nchan + nt - 1) / nt, nbl);
  k_cell_table<<<g2, nt, 0, s>>>(d_freq, d_uvw, nchan, nbl, du, dv, d_cells);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}
