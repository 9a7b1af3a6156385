// Per-image statistics, S/N threshold and candidate list (Law et al. 2018,
// section 3.1: point sources with S/N above a threshold, typically 6 sigma,
// go to the candidate database).
//
// One workgroup per image.  Pass 1 finds the signed peak (ties: lowest
// y*N + x) and histograms the top 11 bits of |img|; passes 2 and 3 refine the
// bin holding the order statistic of rank floor((N*N - 1) / 2) on the next 11
// and the last 9 bits.  For non-negative IEEE floats the bit pattern orders
// like the value, so the three bins name the exact lower median.  sigma is
// that median times a scale: 1.4826 for the images of the transient search
// (MAD about zero of a Gaussian), 1/sqrt(2 ln 2) for the amplitude images of
// the periodicity search (the Rayleigh median).
#include "rf_internal.h"

namespace {

constexpr int kNT = 1024;
constexpr int kWaves = kNT / 64;
constexpr int kBins = 2048;

struct Best {
  float v;
  int i;
};

__device__ __forceinline__ bool better(float v, int i, float bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// Exclusive prefix sum over the workgroup (64-wide wavefronts).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < kWaves ? wsum[lane] : 0u;
    uint32_t winc = w;
#pragma unroll
    for (int o = 1; o < kWaves; o <<= 1) {
      const uint32_t y = __shfl_up(winc, o, 64);
      if (lane >= o) winc += y;
    }
    if (lane < kWaves) wsum[lane] = winc - w;
  }
  __syncthreads();
  const uint32_t r = inc - x + wsum[wid];
  __syncthreads();
  return r;
}

// Given hist[kBins] and a rank, find the bin holding it; writes (bin, rank
// within bin) to sel[0..1].  kBins == 2 * kNT: each thread owns two bins.
__device__ __forceinline__ void select_bin(const uint32_t *hist, uint32_t rank, uint32_t *wsum,
                                           uint32_t *sel) {
  const int t = threadIdx.x;
  const uint32_t h0 = hist[2 * t], h1 = hist[2 * t + 1];
  const uint32_t pre = block_exclusive_scan(h0 + h1, wsum);
  if (rank >= pre && rank < pre + h0 + h1) {
    if (rank < pre + h0) {
      sel[0] = 2 * t;
      sel[1] = rank - pre;
    } else {
      sel[0] = 2 * t + 1;
      sel[1] = rank - pre - h0;
    }
  }
  __syncthreads();
}

template <bool kGen>
__global__ __launch_bounds__(kNT) void k_search(const float *__restrict__ img, int npix,
                                               const rf_image_tag *__restrict__ tags,
                                               rf_tag_gen gen, rf_image_stats *__restrict__ stats,
                                               rf_candidate *__restrict__ cand, int cap,
                                               int32_t *__restrict__ ncand, float thr,
                                               int t_begin, int t_end, float sigma_scale) {
  __shared__ uint32_t hist[kBins];
  __shared__ uint32_t wsum[kWaves];
  __shared__ uint32_t sel[2];
  __shared__ float bv_s[kWaves];
  __shared__ int bi_s[kWaves];
  const int n = blockIdx.x;
  const int tid = threadIdx.x;
  const size_t np2 = (size_t)npix * npix;
  const float4 *im4 = reinterpret_cast<const float4 *>(img + (size_t)n * np2);
  const int n4 = (int)(np2 / 4);
  const uint32_t rank = (uint32_t)((np2 - 1) / 2);

  for (int i = tid; i < kBins; i += kNT) hist[i] = 0;
  __syncthreads();

  // pass 1: peak and top-11-bit histogram of |x|
  float bv = -__builtin_inff();
  int bi = 0x7fffffff;
  for (int q = tid; q < n4; q += kNT) {
    const float4 v = im4[q];
    const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (better(e[c], 4 * q + c, bv, bi)) {
        bv = e[c];
        bi = 4 * q + c;
      }
      const uint32_t key = __float_as_uint(e[c]) & 0x7fffffffu;
      atomicAdd(&hist[key >> 20], 1u);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (better(ov, oi, bv, bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if ((tid & 63) == 0) {
    bv_s[tid >> 6] = bv;
    bi_s[tid >> 6] = bi;
  }
  __syncthreads();
  select_bin(hist, rank, wsum, sel);
  const uint32_t b1 = sel[0];
  uint32_t r1 = sel[1];
  __syncthreads();

  // pass 2: bits 19..9 inside bin b1
  for (int i = tid; i < kBins; i += kNT) hist[i] = 0;
  __syncthreads();
  for (int q = tid; q < n4; q += kNT) {
    const float4 v = im4[q];
    const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t key = __float_as_uint(e[c]) & 0x7fffffffu;
      if ((key >> 20) == b1) atomicAdd(&hist[(key >> 9) & 2047u], 1u);
    }
  }
  __syncthreads();
  select_bin(hist, r1, wsum, sel);
  const uint32_t pre2 = (b1 << 11) | sel[0];
  r1 = sel[1];
  __syncthreads();

  // pass 3: bits 8..0 inside (b1, b2)
  for (int i = tid; i < kBins; i += kNT) hist[i] = 0;
  __syncthreads();
  for (int q = tid; q < n4; q += kNT) {
    const float4 v = im4[q];
    const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t key = __float_as_uint(e[c]) & 0x7fffffffu;
      if ((key >> 9) == pre2) atomicAdd(&hist[key & 511u], 1u);
    }
  }
  __syncthreads();
  select_bin(hist, r1, wsum, sel);

  if (tid == 0) {
    float pv = bv_s[0];
    int pi = bi_s[0];
    for (int w = 1; w < kWaves; ++w)
      if (better(bv_s[w], bi_s[w], pv, pi)) {
        pv = bv_s[w];
        pi = bi_s[w];
      }
    const float med = __uint_as_float((pre2 << 9) | sel[0]);
    const float sigma = sigma_scale * med;
    const float snr = sigma > 0.f ? pv / sigma : 0.f;
    const int x = pi % npix, y = pi / npix;
    if (stats) {
      rf_image_stats st;
      st.peak = pv;
      st.sigma = sigma;
      st.snr = snr;
      st.x = x;
      st.y = y;
      stats[n] = st;
    }
    rf_image_tag tg;
    if (kGen) {
      tg.dm_idx = gen.dm_idx;
      tg.width_idx = gen.width_idx;
      tg.t_int = (gen.k0 + n) * gen.width;
    } else {
      tg = tags[n];
    }
    if (snr > thr && tg.t_int >= t_begin && tg.t_int < t_end) {
      const int slot = atomicAdd(ncand, 1);
      if (slot < cap) {
        rf_candidate c;
        c.dm_idx = tg.dm_idx;
        c.width_idx = tg.width_idx;
        c.t_int = tg.t_int;
        c.x = x;
        c.y = y;
        c.snr = snr;
        c.peak = pv;
        c.sigma = sigma;
        cand[slot] = c;
      }
    }
  }
}

__global__ void k_zero_i32(int32_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

rf_status launch_zero_i32(int32_t *p, int n, hipStream_t s) {
  if (n <= 0) return RF_OK;
  k_zero_i32<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

rf_status launch_search_ex(const rf_plan *p, const float *img, int nimg,
                           const rf_image_tag *tags, const rf_tag_gen *gen, rf_image_stats *stats,
                           rf_candidate *cand, int cap, int32_t *ncand, float sigma_scale,
                           int t_begin, int t_end, hipStream_t s) {
  if (nimg <= 0) return RF_OK;
  if (gen) {
    k_search<true><<<nimg, kNT, 0, s>>>(img, p->npix, nullptr, *gen, stats, cand, cap, ncand,
                                        p->threshold, t_begin, t_end, sigma_scale);
  } else {
    rf_tag_gen none{0, 0, 1, 0};
    k_search<false><<<nimg, kNT, 0, s>>>(img, p->npix, tags, none, stats, cand, cap, ncand,
                                         p->threshold, t_begin, t_end, sigma_scale);
  }
  RF_HIP_TRY(hipGetLastError());
  return RF_OK;
}

rf_status launch_search(const rf_plan *p, const float *img, int nimg, const rf_image_tag *tags,
                        const rf_tag_gen *gen, rf_image_stats *stats, rf_candidate *cand,
                        int cap, int32_t *ncand, hipStream_t s) {
  return launch_search_ex(p, img, nimg, tags, gen, stats, cand, cap, ncand, 1.4826f, p->t_begin,
                          p->t_end, s);
}
