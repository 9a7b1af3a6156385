// Streaming kernels over the segment: dedispersion and boxcar resampling.
//
// Dedispersion in the visibility domain (Law et al. 2018, section 2.2) is a
// pure gather: every output element is one input element shifted in time by
// its channel's integer delay, or zero past the end of the segment.  Threads
// run along the contiguous (baseline, channel) axis so both the reads (one
// channel-run per delay value) and the writes are coalesced 16-byte accesses;
// each thread walks a chunk of integrations so a channel's delay is loaded
// once.
//
// Resampling (Figure 2's loop over sampling times) is a decimating boxcar mean
// accumulated in float32 in increasing sample order and scaled by the float
// reciprocal of the width (exact for powers of two).
//
// Mean subtraction (section 3.1: the mean visibility in time is subtracted on
// timescales below the fringe rate, which removes constant sources) works in
// place on the segment: a thread owns one (baseline, channel, polarisation)
// value, sums it over the segment in float64 with U loads in flight, then
// subtracts the mean from every integration; CF16 storage is rounded back to
// nearest even.
#include "rf_internal.h"

#include <hip/hip_fp16.h>

namespace {

constexpr int kThreads = 256;
constexpr int kTChunk = 32;

template <typename E>
__global__ __launch_bounds__(kThreads) void k_dedisperse(const E *__restrict__ in,
                                                         E *__restrict__ out,
                                                         const int32_t *__restrict__ delay,
                                                         int nint, int nbc, int nchan) {
  const int bc = blockIdx.x * kThreads + threadIdx.x;
  if (bc >= nbc) return;
  const int d = delay[bc % nchan];
  const int t0 = blockIdx.y * kTChunk;
  const int t1 = min(nint, t0 + kTChunk);
  const size_t plane = (size_t)nbc;
  E zero;
  __builtin_memset(&zero, 0, sizeof(E));
  constexpr int U = 8;  // loads in flight per thread
  for (int tb = t0; tb < t1; tb += U) {
    E v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {  // branch-free: clamp the address, zero the value
      const int src = tb + u + d;
      const E x = in[(size_t)min(src, nint - 1) * plane + bc];
      v[u] = src < nint ? x : zero;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (tb + u < t1) out[(size_t)(tb + u) * plane + bc] = v[u];
  }
}

__device__ __forceinline__ float2 load_c(const float2 *p, size_t i) { return p[i]; }
__device__ __forceinline__ float2 load_c(const __half2 *p, size_t i) {
  return __half22float2(p[i]);
}

template <typename Ein>
__global__ __launch_bounds__(kThreads) void k_resample(const Ein *__restrict__ in,
                                                       float2 *__restrict__ out, int nout,
                                                       int width, int nelem) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= nelem) return;
  const int k0 = blockIdx.y * kTChunk;
  const int k1 = min(nout, k0 + kTChunk);
  const float iw = 1.0f / (float)width;  // exact for powers of two
  for (int k = k0; k < k1; ++k) {
    const size_t base = (size_t)k * width * nelem + e;
    float2 acc = make_float2(0.f, 0.f);
    for (int j = 0; j < width; ++j) {
      const float2 x = load_c(in, base + (size_t)j * nelem);
      acc.x += x.x;
      acc.y += x.y;
    }
    out[(size_t)k * nelem + e] = make_float2(acc.x * iw, acc.y * iw);
  }
}

__device__ __forceinline__ void store_c(float2 *p, size_t i, float2 v) { p[i] = v; }
__device__ __forceinline__ void store_c(__half2 *p, size_t i, float2 v) {
  p[i] = __float22half2_rn(v);
}

template <typename E>
__global__ __launch_bounds__(kThreads) void k_mean_subtract(E *__restrict__ vis, int nint,
                                                            int nelem) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= nelem) return;
  constexpr int U = 8;
  double sr = 0.0, si = 0.0;
  for (int t0 = 0; t0 < nint; t0 += U) {
    float2 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      x[u] = load_c(vis, (size_t)min(t0 + u, nint - 1) * nelem + e);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (t0 + u < nint) {
        sr += (double)x[u].x;
        si += (double)x[u].y;
      }
  }
  const float2 m = make_float2((float)(sr / nint), (float)(si / nint));
  for (int t0 = 0; t0 < nint; t0 += U) {
    float2 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      x[u] = load_c(vis, (size_t)min(t0 + u, nint - 1) * nelem + e);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (t0 + u < nint)
        store_c(vis, (size_t)(t0 + u) * nelem + e, make_float2(x[u].x - m.x, x[u].y - m.y));
  }
}

}  // namespace

rf_status launch_mean_subtract(const rf_plan *p, void *vis, hipStream_t s) {
  const int nelem = p->nbl * p->nchan * p->npol;  // complex values per integration
  const dim3 grid((nelem + kThreads - 1) / kThreads);
  if (p->vis_dtype == RF_CF32)
    k_mean_subtract<float2><<<grid, kThreads, 0, s>>>((float2 *)vis, p->nint, nelem);
  else
    k_mean_subtract<__half2><<<grid, kThreads, 0, s>>>((__half2 *)vis, p->nint, nelem);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

rf_status launch_dedisperse(const rf_plan *p, const int32_t *d_delay_row, const void *in,
                            void *out, hipStream_t s) {
  const int nbc = p->nbl * p->nchan;
  dim3 grid((nbc + kThreads - 1) / kThreads, (p->nint + kTChunk - 1) / kTChunk);
  const int ebytes = p->npol * (p->vis_dtype == RF_CF32 ? 8 : 4);
  switch (ebytes) {
    case 16:
      k_dedisperse<uint4><<<grid, kThreads, 0, s>>>((const uint4 *)in, (uint4 *)out,
                                                    d_delay_row, p->nint, nbc, p->nchan);
      break;
    case 8:
      k_dedisperse<uint2><<<grid, kThreads, 0, s>>>((const uint2 *)in, (uint2 *)out,
                                                    d_delay_row, p->nint, nbc, p->nchan);
      break;
    default:
      k_dedisperse<uint32_t><<<grid, kThreads, 0, s>>>((const uint32_t *)in, (uint32_t *)out,
                                                       d_delay_row, p->nint, nbc, p->nchan);
      break;
  }
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

rf_status launch_resample(const rf_plan *p, int width, const void *in, int in_dtype, int nin,
                          float2 *out, hipStream_t s) {
  const int nout = nin / width;
  if (nout == 0) return RF_OK;
  const int nelem = p->nbl * p->nchan * p->npol;  // complex numbers per integration
  dim3 grid((nelem + kThreads - 1) / kThreads, (nout + kTChunk - 1) / kTChunk);
  if (in_dtype == RF_CF32)
    k_resample<float2><<<grid, kThreads, 0, s>>>((const float2 *)in, out, nout, width, nelem);
  else
    k_resample<__half2><<<grid, kThreads, 0, s>>>((const __half2 *)in, out, nout, width, nelem);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}
