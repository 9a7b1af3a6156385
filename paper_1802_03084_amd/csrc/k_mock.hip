// Synthetic data on the device: counter-based Gaussian noise and mock
// transients.
//
// Mock transients (Law et al. 2018, section 3.3: the pipeline inserts mock
// sources into calibrated data to measure its efficiency and sensitivity) are
// dispersed boxcar point sources added to a segment in place.  One thread owns
// one (baseline, channel) pair and adds every mock of a launch, in order, to
// the integrations the mock's sweep touches in that channel, so no two threads
// write the same value and a value is rounded once per mock.  The arrival lag
// (section 2.1 footnote, cold-plasma law) and the fringe phase are float64
// arguments, evaluated one IEEE operation at a time with contraction off; only
// the sum with the stored value is rounded, to float32 or, for float16
// storage, to nearest even through a round-to-odd float32 step (float32 keeps
// more than 11 + 2 bits, so the two roundings equal one direct rounding).
//
// Noise: complex element e of a stream takes Philox4x32-10 block e / 2
// (counter (e/2 mod 2^32, e/2 div 2^32, stream, 0), key = the 64-bit seed;
// Salmon et al. 2011) and turns two of its words into one Box-Muller pair
// (Box and Muller 1958) in float64, rounded to float32; float16 storage rounds
// those float32 values to nearest even.  Any element can be regenerated from
// its index alone, so overlapping windows of one stream hold the same values.
#pragma clang fp contract(off)

#include "rf_internal.h"

#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>

namespace {

constexpr int kThreads = 256;
constexpr double kTwoPi = 6.283185307179586;  // float64 nearest to 2 pi
constexpr double kLight = 299792458.0;        // m/s

// ---------------------------------------------------------------- Philox4x32-10

struct U4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c.x0), lo0 = M0 * c.x0;
    const uint32_t hi1 = __umulhi(M1, c.x2), lo1 = M1 * c.x2;
    c = U4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

__device__ __forceinline__ float2 box_muller(uint32_t a, uint32_t b) {
  const double u1 = ((double)a + 0.5) * 0x1p-32;
  const double u2 = ((double)b + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(kTwoPi * u2, &s, &c);
  return make_float2((float)(r * c), (float)(r * s));
}

__device__ __forceinline__ void put(float2 *p, int64_t i, float2 v) { p[i] = v; }
__device__ __forceinline__ void put(__half2 *p, int64_t i, float2 v) {
  p[i] = __float22half2_rn(v);
}

template <typename E>
__global__ __launch_bounds__(kThreads) void k_noise(E *__restrict__ out, int64_t e_first,
                                                    int64_t n_elem, uint32_t k0, uint32_t k1,
                                                    uint32_t stream) {
  const int64_t n0 = e_first >> 1;
  const int64_t n1 = (e_first + n_elem - 1) >> 1;  // last block, inclusive
  const int64_t step = (int64_t)gridDim.x * kThreads;
  for (int64_t n = n0 + (int64_t)blockIdx.x * kThreads + threadIdx.x; n <= n1; n += step) {
    const U4 x = philox4x32_10(U4{(uint32_t)n, (uint32_t)((uint64_t)n >> 32), stream, 0u}, k0, k1);
    const int64_t e = 2 * n;
    if (e >= e_first) put(out, e - e_first, box_muller(x.x0, x.x1));
    if (e + 1 < e_first + n_elem) put(out, e + 1 - e_first, box_muller(x.x2, x.x3));
  }
}

// ---------------------------------------------------------------- injection

struct MockPack {
  int32_t n, pad;
  rf_mock m[kMocksPerLaunch];
};

// float64 -> float16 rounded to nearest even: round to odd in float32
// (truncate, then set the last bit if anything was cut off), then round to
// nearest even in float16.
__device__ __forceinline__ __half half_rn(double x) {
  float f = __double2float_rz(x);
  if ((double)f != x) f = __uint_as_float(__float_as_uint(f) | 1u);
  return __float2half_rn(f);
}

__device__ __forceinline__ void add_store(float2 *p, int64_t i, double re, double im) {
  const float2 o = p[i];
  p[i] = make_float2((float)((double)o.x + re), (float)((double)o.y + im));
}
__device__ __forceinline__ void add_store(__half2 *p, int64_t i, double re, double im) {
  const float2 o = __half22float2(p[i]);
  __half2 v;
  v.x = half_rn((double)o.x + re);
  v.y = half_rn((double)o.y + im);
  p[i] = v;
}

template <typename E>
__global__ __launch_bounds__(kThreads) void k_inject(E *__restrict__ vis,
                                                     const double *__restrict__ freq,
                                                     const double *__restrict__ uvw, int nint,
                                                     int nbl, int nchan, int npol, double nu_top,
                                                     double tint_s, double kdm, double t_first,
                                                     MockPack pk) {
  const int bc = blockIdx.x * kThreads + threadIdx.x;
  if (bc >= nbl * nchan) return;
  const int b = bc / nchan, c = bc - b * nchan;
  const double nu = freq[c];
  const double inv = 1.0 / (nu * nu);
  const double inv_top = 1.0 / (nu_top * nu_top);
  const double f_hz = nu * 1e9;
  const double u_l = (uvw[3 * b + 0] * f_hz) / kLight;
  const double v_l = (uvw[3 * b + 1] * f_hz) / kLight;
  for (int k = 0; k < pk.n; ++k) {
    const rf_mock mk = pk.m[k];
    const double lag = (kdm * mk.dm) * (inv - inv_top);
    const double start = mk.t0 + lag / tint_s;
    const double end = start + mk.width;
    // absolute integrations t_first .. t_first + nint - 1 are in the buffer
    const double js = fmax(floor(start), t_first);
    const double je = fmin(ceil(end), t_first + (double)nint);
    if (!(js < je)) continue;
    const double phase = -(kTwoPi * (u_l * mk.l + v_l * mk.m));
    double sn, cs;
    sincos(phase, &sn, &cs);
    const int j0 = (int)(js - t_first), j1 = (int)(je - t_first);
    for (int j = j0; j < j1; ++j) {
      const double t = t_first + (double)j;
      const double frac = fmin(t + 1.0, end) - fmax(t, start);
      if (!(frac > 0.0)) continue;
      const double s = mk.amp * frac;
      const double re = s * cs, im = s * sn;
      const int64_t base = ((int64_t)j * nbl + b) * nchan + c;
      for (int p = 0; p < npol; ++p) add_store(vis, base * npol + p, re, im);
    }
  }
}

}  // namespace

rf_status launch_noise(const rf_plan *p, uint64_t seed, uint32_t stream, int64_t t_first,
                       void *vis, hipStream_t s) {
  const int64_t per = (int64_t)p->nbl * p->nchan * p->npol;
  const int64_t n_elem = per * p->nint;
  if (n_elem == 0) return RF_OK;
  const int64_t nblk = ((t_first * per + n_elem - 1) >> 1) - ((t_first * per) >> 1) + 1;
  const int64_t want = (nblk + kThreads - 1) / kThreads;
  const int grid = (int)std::min<int64_t>(want, 65536);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (p->vis_dtype == RF_CF32)
    k_noise<float2><<<grid, kThreads, 0, s>>>((float2 *)vis, t_first * per, n_elem, k0, k1, stream);
  else
    k_noise<__half2><<<grid, kThreads, 0, s>>>((__half2 *)vis, t_first * per, n_elem, k0, k1,
                                               stream);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

rf_status launch_inject(const rf_plan *p, const rf_mock *mocks, int nmock, int64_t t_first,
                        void *vis, hipStream_t s) {
  const int nbc = p->nbl * p->nchan;
  if (nbc == 0 || p->nint == 0) return RF_OK;
  const double nu_top = *std::max_element(p->freq.begin(), p->freq.end());
  const int grid = (nbc + kThreads - 1) / kThreads;
  for (int k0 = 0; k0 < nmock; k0 += kMocksPerLaunch) {
    MockPack pk{};
    pk.n = std::min(kMocksPerLaunch, nmock - k0);
    for (int k = 0; k < pk.n; ++k) pk.m[k] = mocks[k0 + k];
    if (p->vis_dtype == RF_CF32)
      k_inject<float2><<<grid, kThreads, 0, s>>>((float2 *)vis, p->d_freq, p->d_uvw, p->nint,
                                                 p->nbl, p->nchan, p->npol, nu_top, p->tint_s,
                                                 p->kdm, (double)t_first, pk);
    else
      k_inject<__half2><<<grid, kThreads, 0, s>>>((__half2 *)vis, p->d_freq, p->d_uvw, p->nint,
                                                  p->nbl, p->nchan, p->npol, nu_top, p->tint_s,
                                                  p->kdm, (double)t_first, pk);
    RF_HIP_TRY(hipGetLastError());
  }
  return RF_OK;
}
