// Fused whole-segment search (Law et al. 2018, section 3.1 and Figure 2):
// per DM trial, one pass over the segment dedisperses, resamples to every
// trial width and forms Stokes I; per pair of images the row pass gathers uv
// cells straight from those samples and transforms the rows; the column pass
// transforms the columns and reduces every image to its peak and to the few
// pixels that can hold the median; a last kernel picks the exact median and
// thresholds.  No dense grid and no image ever reaches HBM.
//
// Exact median without the image: the image rms is known before the column
// pass (Parseval: sum img^2 = N^2 / W^2 * sum |H|^2 over the Hermitian part
// H of the grid), and for noise images median|img| / rms sits within 0.2 %
// of 0.6745.  The column pass therefore counts pixels below a bracket
// 0.6745 rms (1 -/+ b, b from 1 % down to 0.4 % as images grow) and keeps
// those inside it; if the rank of the lower
// median falls inside the bracket the kept values contain it and the result
// is exact.  Otherwise (a bright source shifts the rms, or a region of kept
// values overflows) the image is recomputed by the step chain after the
// segment, so every reported sigma is the exact lower median.
//
// Every value is computed with the same operations in the same order as the
// step chain (rf_dedisperse -> rf_resample -> rf_grid -> rf_image ->
// rf_search), so both paths give bit-identical images.
#include "rf_internal.h"
#include "fft.h"

#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <numeric>
#include <vector>

namespace {

using namespace rf;

constexpr int kMaxLanes = 4;           // concurrent batch pipelines (streams) of a segment search
constexpr int kMaxW = 8;               // widths handled by one pass over the segment
constexpr float kMedOverRms = 0.6745f; // median |x| / rms of a zero-mean Gaussian
// half-width of the median bracket (relative): the bracket holds about 0.86%
// of the pixels per percent of half-width; larger images have a tighter
// median/rms ratio (0.12% spread at 1024^2) and get a narrower bracket, so
// that fewer values are kept (measured on the survey search: 0.7% at 1024^2
// 1.1% faster than 1% with no exact fallbacks; 0.5% sent 46 of 491,520
// noise images to the fallback and was 9% slower)
template <int N>
constexpr float bracket_of() { return N >= 2048 ? 0.004f : (N >= 1024 ? 0.007f : 0.01f); }
constexpr int kDrsThreads = 256;
constexpr int kSelThreads = 512;
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct WidthSet {
  int w[kMaxW];
  int nk[kMaxW];     // images of each width (= nint / w)
  float2 *out[kMaxW];
  int nw;
};

constexpr int kMaxColWaves = 8;  // waves of a column workgroup, at most

struct ColPart {   // per (image, column workgroup)
  float maxv;
  int32_t maxi;
  uint32_t cnt_lo;  // pixels with |value| below the bracket
  float lo, hi;     // the bracket [lo, hi) (identical in every workgroup of a pair)
  // pixels inside the bracket found by each wave of the workgroup; wave w
  // keeps min(nw[w], capb / waves) of their values in its part of the tile's
  // list region (values beyond it send the image to the exact fallback)
  uint32_t nw[kMaxColWaves];
};

__device__ __forceinline__ bool better(float v, int i, float bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// Cross-lane exchange with lane ^ o (o < 64): one ds_bpermute on the byte
// address ((lane ^ o) << 2), which every exchange at the same o shares.
__device__ __forceinline__ int xaddr(int o) {
  return (int)((__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)) ^ (uint32_t)o)
               << 2);
}
__device__ __forceinline__ float xshfl(float v, int addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ int xshfl(int v, int addr) { return __builtin_amdgcn_ds_bpermute(addr, v); }

// ------------------------------------------------------------------ drs
__device__ __forceinline__ void load_pols(const float2 *vis, size_t e, int P, float2 &a,
                                          float2 &b) {
  if (P == 2) {
    const float4 x = *reinterpret_cast<const float4 *>(vis + 2 * e);
    a = make_float2(x.x, x.y);
    b = make_float2(x.z, x.w);
  } else {
    a = vis[e];
  }
}
__device__ __forceinline__ void load_pols(const __half2 *vis, size_t e, int P, float2 &a,
                                          float2 &b) {
  if (P == 2) {
    const uint2 x = *reinterpret_cast<const uint2 *>(vis + 2 * e);
    a = __half22float2(*reinterpret_cast<const __half2 *>(&x.x));
    b = __half22float2(*reinterpret_cast<const __half2 *>(&x.y));
  } else {
    a = __half22float2(vis[e]);
  }
}

// Dedisperse + boxcar-resample to every width in `ws` + Stokes I, one thread
// per (baseline, channel) walking a chunk of integrations that starts at a
// multiple of every width and holds an even number of each width's images.
// Sums run per polarisation in increasing time and are scaled by 1/w (the
// float reciprocal, exact for powers of two) before the polarisations are
// averaged, exactly as rf_resample followed by rf_grid's Stokes I.  Output
// per width, by image pair (the pairs of the paired transform):
// VI_w[k / 2][bc][k % 2], one 16-byte store per pair, coalesced along bc; the
// odd last image of a width is paired with zeros.
template <typename Ein, int P>
__global__ __launch_bounds__(kDrsThreads) void k_drs(const Ein *__restrict__ vis,
                                                     const int32_t *__restrict__ delay, int nint,
                                                     int nbc, int nchan, int tchunk, WidthSet ws) {
  const int bc = blockIdx.x * kDrsThreads + threadIdx.x;
  if (bc >= nbc) return;
  const int d = delay[bc % nchan];
  const int t0 = blockIdx.y * tchunk;
  const int t1 = min(nint, t0 + tchunk);
  float2 a0[kMaxW], a1[kMaxW], held[kMaxW];  // held: first image of the open pair
  int cnt[kMaxW], kout[kMaxW];
  float inv[kMaxW];  // 1/w: exact for powers of two, so the product is the quotient
#pragma unroll
  for (int j = 0; j < kMaxW; ++j) {
    a0[j] = make_float2(0.f, 0.f);
    a1[j] = a0[j];
    held[j] = a0[j];
    cnt[j] = 0;
    inv[j] = j < ws.nw ? 1.0f / (float)ws.w[j] : 0.f;
    kout[j] = j < ws.nw ? t0 / ws.w[j] : 0;  // even: t0 is an even multiple of every width
  }
  // each sample is read once, batches later: stream it past the caches
  typedef float f4v __attribute__((ext_vector_type(4)));
  auto put = [&](int j, float2 x, float2 y) {
    const f4v v = {x.x, x.y, y.x, y.y};
    __builtin_nontemporal_store(
        v, reinterpret_cast<f4v *>(&ws.out[j][((size_t)(kout[j] >> 1) * nbc + bc) * 2]));
  };
  constexpr int U = 8;  // integrations loaded ahead: U loads in flight per thread
  for (int tb = t0; tb < t1; tb += U) {
    float2 w0[U], w1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {  // branch-free: clamp the address, zero the value
      const int src = tb + u + d;
      float2 a, b = make_float2(0.f, 0.f);
      load_pols(vis, (size_t)min(src, nint - 1) * nbc + bc, P, a, b);
      const bool ok = src < nint;
      w0[u] = ok ? a : make_float2(0.f, 0.f);
      w1[u] = ok ? b : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = tb + u;
      if (t >= t1) break;
      const float2 v0 = w0[u], v1 = w1[u];
#pragma unroll
      for (int j = 0; j < kMaxW; ++j) {
        if (j < ws.nw) {
          a0[j].x += v0.x;
          a0[j].y += v0.y;
          if (P == 2) {
            a1[j].x += v1.x;
            a1[j].y += v1.y;
          }
          if (++cnt[j] == ws.w[j]) {
            const float iw = inv[j];
            float2 vi;
            if (P == 2) {
              const float r0x = a0[j].x * iw, r0y = a0[j].y * iw;
              const float r1x = a1[j].x * iw, r1y = a1[j].y * iw;
              vi = make_float2((r0x + r1x) * 0.5f, (r0y + r1y) * 0.5f);
            } else {
              vi = make_float2(a0[j].x * iw, a0[j].y * iw);
            }
            if (kout[j] & 1)  // uniform: every thread of the workgroup shares t0
              put(j, held[j], vi);
            else
              held[j] = vi;
            ++kout[j];
            a0[j] = make_float2(0.f, 0.f);
            a1[j] = a0[j];
            cnt[j] = 0;
          }
        }
      }
    }
  }
  // a chunk cut short by the end of the segment can close on the first image
  // of a pair: the width's last image, paired with zeros
#pragma unroll
  for (int j = 0; j < kMaxW; ++j)
    if (j < ws.nw && (kout[j] & 1)) put(j, held[j], make_float2(0.f, 0.f));
}

// ------------------------------------------------------------------ rows
// Gridding as a gather: CV[i][c] = sum of the Stokes I samples of uv cell c
// for image i of a batch, in the plan's contributor order (the same sums as
// rf_grid).  A workgroup takes a block of whole cells (at most 1024
// contributors) for one image pair: it stages the block's samples in LDS
// with all loads in flight (one 16-byte load per contributor: the two images
// of a pair sit side by side), then one thread per cell sums them in
// contributor order.  Output by pair: CV[p][c] = (image 2p, image 2p + 1).
// All blocks of one pair run on one XCD (blocks are dealt to the eight XCDs
// round robin), so the pair's samples stay in that XCD's L2; a batch of fewer
// than eight pairs spreads each pair's blocks over 8 / pairs XCDs instead.
constexpr int kCellThreads = 256;
constexpr int kCellPairs = 1;      // image pairs per workgroup (2: 11.0 us, 4: 15.1 us against 9.6 us per survey batch)

__global__ __launch_bounds__(kCellThreads) void k_cellsum(
    const float4 *__restrict__ vi, int nbc, int p0, int npair, int n_cells, int n_cblk,
    const int4 *__restrict__ cblk, const int32_t *__restrict__ coff,
    const int32_t *__restrict__ contrib, float4 *__restrict__ cv, int rep) {
  constexpr int CP = kCellPairs;
  __shared__ float4 val[CP][kCellBlock];
  const int b = blockIdx.x, xcd = b & 7, local = b >> 3;
  int g, blk;  // group of CP image pairs within the batch, cell block
  const int ngrp = (npair + CP - 1) / CP;
  if (rep == 1) {  // at least eight groups: every block of a group on one XCD
    g = (local / n_cblk) * 8 + xcd;
    blk = local % n_cblk;
  } else {  // fewer groups: `rep` XCDs share a group's blocks
    g = xcd / rep;
    blk = local * rep + xcd % rep;
    if (blk >= n_cblk) return;
  }
  if (g >= ngrp) return;
  const int tid = threadIdx.x;
  // the group's pairs; a missing last pair reads the first again and is not stored
  const float4 *v[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) v[c] = vi + (size_t)(p0 + min(g * CP + c, npair - 1)) * nbc;
  // the block's cells and contributor run in one load: one level of
  // dependent loads fewer before the gather
  const int4 bk = cblk[blk];
  const int c0 = bk.x, c1 = bk.y, q0 = bk.z, q1 = bk.w, nq = q1 - q0;
  auto add = [](float4 &acc, const float4 y) {
    acc.x += y.x;
    acc.y += y.y;
    acc.z += y.z;
    acc.w += y.w;
  };
  auto put = [&](int c, int cell, const float4 &acc) {
    if (g * CP + c < npair) cv[(size_t)(g * CP + c) * n_cells + cell] = acc;
  };
  if (nq <= kCellBlock) {
    // stage the block's samples: every index load, then every value load, in
    // flight together.  Every slot of the stage is written (slots past the
    // block hold a copy of its last sample and are never summed), so no
    // branch separates a load from its use and none waits for another.
    constexpr int T = kCellBlock / kCellThreads;
    int bq[T];
#pragma unroll
    for (int t = 0; t < T; ++t) bq[t] = contrib[min(q0 + tid + t * kCellThreads, q1 - 1)];
    // the contributor range of this thread's first cell, fetched alongside
    const int cf = min(c0 + tid, c1 - 1);
    int f0 = coff[cf], f1 = coff[cf + 1];
    float4 x[CP][T];
#pragma unroll
    for (int c = 0; c < CP; ++c)
#pragma unroll
      for (int t = 0; t < T; ++t) x[c][t] = v[c][bq[t]];
#pragma unroll
    for (int c = 0; c < CP; ++c)
#pragma unroll
      for (int t = 0; t < T; ++t) val[c][tid + t * kCellThreads] = x[c][t];
    asm volatile("" ::"v"(f0), "v"(f1));  // keeps the range load ahead of the barrier
    __syncthreads();
    for (int cell = c0 + tid; cell < c1; cell += kCellThreads) {
      if (cell != c0 + tid) {
        f0 = coff[cell];
        f1 = coff[cell + 1];
      }
      float4 acc[CP];
#pragma unroll
      for (int c = 0; c < CP; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
      const int e = f1 - q0;
      int q = f0 - q0;
      // four reads per pair in flight, then the adds in contributor order
      for (; q + 4 <= e; q += 4) {
        float4 y[CP][4];
#pragma unroll
        for (int c = 0; c < CP; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) y[c][k] = val[c][q + k];
#pragma unroll
        for (int c = 0; c < CP; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) add(acc[c], y[c][k]);
      }
      for (; q < e; ++q)
#pragma unroll
        for (int c = 0; c < CP; ++c) add(acc[c], val[c][q]);
#pragma unroll
      for (int c = 0; c < CP; ++c) put(c, cell, acc[c]);
    }
  } else {
    // a cell with more contributors than a block: direct gather, same order
    for (int cell = c0 + tid; cell < c1; cell += kCellThreads) {
      float4 acc[CP];
#pragma unroll
      for (int c = 0; c < CP; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
      const int e = coff[cell + 1];
      for (int q = coff[cell]; q < e; ++q) {
        const int bcq = contrib[q];
#pragma unroll
        for (int c = 0; c < CP; ++c) add(acc[c], v[c][bcq]);
      }
#pragma unroll
      for (int c = 0; c < CP; ++c) put(c, cell, acc[c]);
    }
  }
}

// Row pass.  A workgroup takes one row pair {v, -v} for a block of PBW image
// pairs: it reads the cell sums of both rows (contiguous in cell order), forms
// Z on both rows (row -v is the conjugate-mirror combination of the same
// cells), transforms the 2 PBW rows and writes them.  It also writes each
// image's share of sum |H|^2 (Parseval) for the median bracket of the column
// pass.
template <int N>
struct RowPairCfg {
  // image pairs per workgroup: ~35 KB of LDS from 1024 up, ~18 KB at 512
  // (256 threads), so that several workgroups per CU interleave their load
  // and transform phases
  static constexpr int PBW = N >= 2048 ? 1 : (N >= 512 ? 2 : 4);
  static constexpr int F = 2 * PBW;              // transforms per workgroup
  static constexpr int NT = F * N / RowFft<N>::R0 < 256 ? 256 : F * N / RowFft<N>::R0;
  static constexpr int STRIDE = RowFft<N>::PADDED;
};

template <int N>
__global__ __launch_bounds__(RowPairCfg<N>::NT) void k_rows_pairs(
    const float4 *__restrict__ cv, int n_cells, int nk, int p0, int pbn,
    const int32_t *__restrict__ rp_row, const int32_t *__restrict__ rp_sa,
    const int32_t *__restrict__ rp_sb, int n_rp, int n_rows, const int32_t *__restrict__ zs_off,
    const int32_t *__restrict__ zs_u, const int32_t *__restrict__ zs_ck,
    const int32_t *__restrict__ zs_cmk, float hw, const float2 *__restrict__ tw,
    float2 *__restrict__ M, float *__restrict__ epart) {
  constexpr int PBW = RowPairCfg<N>::PBW, F = RowPairCfg<N>::F, NT = RowPairCfg<N>::NT;
  constexpr int S = RowPairCfg<N>::STRIDE, PS = RowFft<N>::PS;
  __shared__ __align__(16) float2 buf[F * S];
  __shared__ float s_e[2 * PBW];
  static_assert((F * S) % 2 == 0, "the LDS buffer is cleared 16 bytes at a time");
  const int rp = blockIdx.x % n_rp;
  const int pb0 = (blockIdx.x / n_rp) * PBW;  // first pair of this block, batch-local
  const int tid = threadIdx.x;
  TwBases<RowFft<N>, F, NT, true> tb;  // twiddle bases of the row transforms
  tb.load(tw, tid);
  const int r = rp_row[rp];
  const int rm = (N - r) & (N - 1);
  const bool two = rm != r;
  for (int i = tid; i < F * S / 2; i += NT)
    reinterpret_cast<float4 *>(buf)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (tid < 2 * PBW) s_e[tid] = 0.f;
  __syncthreads();
  const int z0 = zs_off[rp], nz = zs_off[rp + 1] - z0;
  // cell sums of this workgroup's pairs, one resource for all of them (a
  // per-lane resource would need a loop over its distinct values)
  const float4 *cvw = cv + (size_t)pb0 * n_cells;
  const uint32_t cvw_bytes = (uint32_t)(max(0, min(PBW, pbn - pb0)) * n_cells) * 16u;
  const float ew = two ? 0.5f : 0.25f;  // |H|^2 = |.|^2/4, counted twice for a row pair
  float e_acc[2 * PBW];                 // this thread's share of each image's energy
#pragma unroll
  for (int q = 0; q < 2 * PBW; ++q) e_acc[q] = 0.f;
  for (int it = tid; it < nz * PBW; it += NT) {
    const int z = z0 + it % nz, pp = it / nz;  // positions fastest: contiguous cells
    const int pl = pb0 + pp;
    if (pl >= pbn) continue;
    const bool hasb = 2 * (p0 + pl) + 1 < nk;
    const int u = zs_u[z], ck = zs_ck[z], cmk = zs_cmk[z];
    // cell sums of images a and b side by side; absent cells read zero
    // through the buffer range check, an absent image b is zero
    const auto rc = buf_rsrc_u(cvw, cvw_bytes);
    const uint32_t pc = (uint32_t)(pp * n_cells);
    const float4 c4 = buf_load_f4(rc, ck >= 0 ? (pc + (uint32_t)ck) * 16u : kNoLoad);
    const float4 m4 = buf_load_f4(rc, cmk >= 0 ? (pc + (uint32_t)cmk) * 16u : kNoLoad);
    const float2 ga = make_float2(c4.x, c4.y), gam = make_float2(m4.x, m4.y);
    const float2 gb = hasb ? make_float2(c4.z, c4.w) : make_float2(0.f, 0.f);
    const float2 gbm = hasb ? make_float2(m4.z, m4.w) : make_float2(0.f, 0.f);
    const float sg = ((r + u) & 1) ? -hw : hw;  // (-1)^(u+v) / (2W)
    buf[pp * S + pidx<PS>(u)] = zval(ga, gam, gb, gbm, sg);
    if (two) buf[(PBW + pp) * S + pidx<PS>((N - u) & (N - 1))] = zval(gam, ga, gbm, gb, sg);
    const float hax = ga.x + gam.x, hay = ga.y - gam.y;
    const float hbx = gb.x + gbm.x, hby = gb.y - gbm.y;
    const float ea = ew * (hax * hax + hay * hay), eb = ew * (hbx * hbx + hby * hby);
#pragma unroll
    for (int q = 0; q < PBW; ++q) {
      e_acc[2 * q] += q == pp ? ea : 0.f;
      e_acc[2 * q + 1] += q == pp ? eb : 0.f;
    }
  }
  // the energy terms: a wave sum per image, then one LDS atomic per wave
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int ad = xaddr(o);
#pragma unroll
    for (int q = 0; q < 2 * PBW; ++q) e_acc[q] += xshfl(e_acc[q], ad);
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 2 * PBW; ++q)
      if (e_acc[q] != 0.f) atomicAdd(&s_e[q], e_acc[q]);
  }
  __syncthreads();
  if (tid < 2 * PBW && pb0 + tid / 2 < pbn)
    epart[((size_t)(pb0 + tid / 2) * n_rp + rp) * 2 + (tid & 1)] = s_e[tid];
  const int sa = rp_sa[rp], sb = rp_sb[rp];
  fft_inverse<RowFft<N>, F, NT, S, true>(
      buf, tb, tid, [&](int f, int i) { return buf[f * S + pidx<PS>(i)]; },
      [&](int f, int x, float2 v) {
        const int side = f / PBW, pp = f % PBW;
        const int pl = pb0 + pp;
        if (pl < pbn && (side == 0 || two))
          M[((size_t)pl * n_rows + (side ? sb : sa)) * N + x] = v;
      });
}

// ------------------------------------------------------------------ columns
// Column pass and per-image statistics.  A workgroup takes a tile of COLS
// adjacent columns of one image pair.  Workgroups are dealt to the eight XCDs
// round robin (b mod 8); XCD x takes a contiguous run of tiles, so the column
// tiles that run together on one XCD are adjacent and share their cache
// lines in that XCD's L2.  All global loads (the tile and the pair's energy
// terms) are issued together, without branches, before any is used.
//
// Per tile and image: the peak (signed max, lowest flat index on ties), the
// count of |pixel| below the median bracket, and the bracket values
// themselves (into this tile's list region of capb values; the count may
// exceed capb, which sends the image to the exact fallback).  The bracket is
// kMedOverRms * rms (1 +- bracket_of<N>()), with the rms from Parseval: the
// image energy is the grid energy (summed by the row pass) over N^2 W^2.
template <int N>
__global__ __launch_bounds__(ColCfg<N>::NT) void k_cols_stats(
    const float2 *__restrict__ M, int n_rows, int vmax, int nimg_w,
    int p0, int pbn, float inv_w, const float2 *__restrict__ tw, const float *__restrict__ epart,
    int n_rp, ColPart *__restrict__ part, float *__restrict__ list, int capb) {
  using Sh = ColFft<N>;
  constexpr int COLS = ColCfg<N>::COLS, NT = ColCfg<N>::NT, S = ColCfg<N>::STRIDE;
  constexpr int CB = N / COLS;
  constexpr int NW = NT / 64;
  constexpr int EPT = ((N / 2 + 1) * 2 + NT - 1) / NT;  // energy terms per thread, at most
  static_assert(NT % 2 == 0, "energy terms alternate a, b by thread parity");
  static_assert(NW <= kMaxColWaves, "per-wave counts of a record");
  __shared__ float2 buf[COLS * S];
  __shared__ float s_e[2][NW];
  __shared__ float w_v[2][NW];
  __shared__ int32_t w_i[2][NW];
  __shared__ uint32_t w_c[2][NW];
  __shared__ uint32_t w_n[2][NW];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int total = pbn * CB;
  const int per = (total + 7) >> 3;  // tiles per XCD
  const int b = blockIdx.x;
  const int L = (b & 7) * per + (b >> 3);
  if ((b >> 3) >= per || L >= total) return;
  const int pl = L / CB, cb = L % CB;
  FirstRegs<Sh, COLS, NT> x;
  TwBases<Sh, COLS, NT, false> tb;  // twiddle bases, loaded with the tile
  {  // rows outside the stored band read as zero through the range check
    const auto rm = buf_rsrc(M + (size_t)pl * n_rows * N + cb * COLS, (uint32_t)n_rows * N * 8u);
    fft_first_load<Sh, COLS, NT, false>(
        tid,
        [&](int f, int i) {
          return buf_load_f2(rm, (uint32_t)(band_slot_raw(i, N, vmax) * N + f) * 8u);
        },
        x);
  }
  tb.load(tw, tid);
  float e = 0.f;  // grid energy of image a (even threads) or b (odd threads)
  {
    const auto re = buf_rsrc(epart + (size_t)pl * n_rp * 2, (uint32_t)n_rp * 8u);
    float ep[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int t = tid + q * NT;
      ep[q] = buf_load_f1(re, t < 2 * n_rp ? (uint32_t)t * 4u : kNoLoad);
    }
    // keep the scheduler from starting the transform before every load is issued
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < EPT; ++q) e += ep[q];
  }
  fft_first_dft<Sh, COLS, NT>(x);
#pragma unroll
  for (int o = 2; o < 64; o <<= 1) e += xshfl(e, xaddr(o));
  fft_first_store<Sh, COLS, NT, S, false>(buf, tb, tid, x);
  if (lane < 2) s_e[lane][wid] = e;
  __syncthreads();
  float ea = 0.f, eb = 0.f;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    ea += s_e[0][w];
    eb += s_e[1][w];
  }
  const float ma = kMedOverRms * (sqrtf(ea) * inv_w), mb = kMedOverRms * (sqrtf(eb) * inv_w);
  const float lo_a = ma * (1.0f - bracket_of<N>()), hi_a = ma * (1.0f + bracket_of<N>());
  const float lo_b = mb * (1.0f - bracket_of<N>()), hi_b = mb * (1.0f + bracket_of<N>());
  const bool hasb = 2 * (p0 + pl) + 1 < nimg_w;
  const int x0 = cb * COLS;
  // This wave's part of the tile's list regions (capb values per image): capw
  // values from wid * capw, filled in order by a wave-uniform running count.
  // (The wave index is made explicitly uniform so that the buffer resources
  // live in scalar registers.)
  const int capw = capb / NW;
  const int uwid = __builtin_amdgcn_readfirstlane(wid);
  const auto rla = buf_rsrc(list + ((size_t)(2 * pl) * CB + cb) * capb + uwid * capw,
                            (uint32_t)capw * 4u);
  const auto rlb = buf_rsrc(list + ((size_t)(2 * pl + 1) * CB + cb) * capb + uwid * capw,
                            (uint32_t)capw * 4u);
  float bva = -__builtin_inff(), bvb = -__builtin_inff();
  int bia = 0x7fffffff, bib = 0x7fffffff;
  uint32_t ca = 0, cbn = 0;  // wave-uniform: pixels below the bracket
  uint32_t na = 0, nb = 0;   // wave-uniform: bracket members found so far
  fft_rest_blocks<Sh, COLS, NT, S, false>(buf, tb, tid, [&](int f, int k0, int ks, auto &v) {
    constexpr int R = sizeof(v) / sizeof(v[0]);
    // Image b is computed even when the pair has no second image: its values
    // are then never used (no record is written for it and no select reads
    // its list region), and the loop stays free of branches.
    //
    // The peak: the butterfly's maximum and the lowest of its outputs that
    // hold it (the outputs ascend in flat index with r), merged into the
    // thread's peak by value, then lower flat index.  The outputs are
    // already image pixels: 1/W is folded into Z.
    {
      float ma = v[0].x, mb = v[0].y;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        ma = fmaxf(ma, v[r].x);
        mb = fmaxf(mb, v[r].y);
      }
      int ra = R - 1, rb = R - 1;
#pragma unroll
      for (int r = R - 2; r >= 0; --r) {
        ra = v[r].x == ma ? r : ra;
        rb = v[r].y == mb ? r : rb;
      }
      const int ia = (k0 + ra * ks) * N + x0 + f, ib = (k0 + rb * ks) * N + x0 + f;
      if (better(ma, ia, bva, bia)) {
        bva = ma;
        bia = ia;
      }
      if (better(mb, ib, bvb, bib)) {
        bvb = mb;
        bib = ib;
      }
    }
    // The median bracket, per output row of the wave: the count below it (a
    // popcount of one ballot) and its members, |p| in [lo, hi) (a second
    // ballot, less the first), written to this wave's list part at the
    // running count plus the members in lower lanes.  Slots at or past capw
    // fall outside the buffer resource and are dropped by the hardware (the
    // count still grows, which sends the image to the exact fallback).  NaN
    // pixels are neither below nor inside the bracket.  The list holds the
    // signed pixel values; the select ranks their magnitudes.
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float pa = v[r].x, pb = v[r].y;
      // ballots of the plain compares (one VALU compare each); the member
      // masks by scalar arithmetic
      const bool a_lo = fabsf(pa) < lo_a, a_hi = fabsf(pa) < hi_a;
      const bool b_lo = fabsf(pb) < lo_b, b_hi = fabsf(pb) < hi_b;
      const uint64_t la = __builtin_amdgcn_ballot_w64(a_lo), lb = __builtin_amdgcn_ballot_w64(b_lo);
      const uint64_t ia = __builtin_amdgcn_ballot_w64(a_hi) & ~la;
      const uint64_t ib = __builtin_amdgcn_ballot_w64(b_hi) & ~lb;
      ca += (uint32_t)__popcll(la);
      cbn += (uint32_t)__popcll(lb);
      if (ia) {
        if (a_hi && !a_lo) {
          const uint32_t below = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(ia >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ia, 0u));
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(pa), rla, (int)((na + below) * 4u),
                                                0, 0);
        }
        na += (uint32_t)__popcll(ia);
      }
      if (ib) {
        if (b_hi && !b_lo) {
          const uint32_t below = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(ib >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ib, 0u));
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(pb), rlb, (int)((nb + below) * 4u),
                                                0, 0);
        }
        nb += (uint32_t)__popcll(ib);
      }
    }
  });
  // Tile peak: (value, flat index) pairs reduced by value, then lower index,
  // over the wave and then the workgroup's waves.
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int ad = xaddr(o);
    const float ova = xshfl(bva, ad), ovb = xshfl(bvb, ad);
    const int oia = xshfl(bia, ad), oib = xshfl(bib, ad);
    if (better(ova, oia, bva, bia)) {
      bva = ova;
      bia = oia;
    }
    if (better(ovb, oib, bvb, bib)) {
      bvb = ovb;
      bib = oib;
    }
  }
  if (lane == 0) {
    w_v[0][wid] = bva;
    w_v[1][wid] = bvb;
    w_i[0][wid] = bia;
    w_i[1][wid] = bib;
    w_c[0][wid] = ca;
    w_c[1][wid] = cbn;
    w_n[0][wid] = na;
    w_n[1][wid] = nb;
  }
  __syncthreads();
  if (tid < 2 && (tid == 0 || hasb)) {
    float pk = w_v[tid][0];
    int i = w_i[tid][0];
    uint32_t c = w_c[tid][0];
    for (int w = 1; w < NW; ++w) {
      if (better(w_v[tid][w], w_i[tid][w], pk, i)) {
        pk = w_v[tid][w];
        i = w_i[tid][w];
      }
      c += w_c[tid][w];
    }
    ColPart cp;
    cp.maxv = pk;
    cp.maxi = i;
    cp.cnt_lo = c;
    cp.lo = tid == 0 ? lo_a : lo_b;
    cp.hi = tid == 0 ? hi_a : hi_b;
#pragma unroll
    for (int w = 0; w < kMaxColWaves; ++w) cp.nw[w] = w < NW ? w_n[tid][w] : 0u;
    part[(size_t)(2 * pl + tid) * CB + cb] = cp;
  }
}

// ------------------------------------------------------------------ select
constexpr int kBins = 2048;
constexpr uint32_t kBinCap = 1024;  // values of one bracket bin ranked directly

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < wid; ++w) add += wsum[w];
  __syncthreads();
  return inc - x + add;
}

// Finds the bin of hist[kBins] that holds `rank`; BPT consecutive bins per
// thread.
__device__ __forceinline__ void sel_bin(const uint32_t *hist, uint32_t rank, uint32_t *wsum,
                                        uint32_t *sel) {
  constexpr int BPT = kBins / kSelThreads;
  static_assert(BPT * kSelThreads == kBins, "bins divide over the threads");
  const int t = threadIdx.x;
  uint32_t h[BPT], tot = 0;
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    h[i] = hist[BPT * t + i];
    tot += h[i];
  }
  uint32_t pre = block_excl_scan(tot, wsum);
  if (rank >= pre && rank < pre + tot) {
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      if (rank >= pre && rank < pre + h[i]) {
        sel[0] = BPT * t + i;
        sel[1] = rank - pre;
      }
      pre += h[i];
    }
  }
  __syncthreads();
}

constexpr int kMaxCB = 512;       // column workgroups per image, at most
// bracket values staged in LDS: about 0.86% of the pixels per percent of
// bracket half-width (6,300 at 1024^2, 14,400 at 2048^2), with room to spare;
// more send the image to the exact fallback
template <int N>
constexpr int lds_vals_of() { return N >= 2048 ? 20480 : (N >= 1024 ? 10240 : 8192); }

// Per image: combines the column workgroups' records (peak, count below the
// bracket, per-wave bracket counts), stages every kept bracket magnitude in
// LDS, and finds the median |value| among them.  Images whose median is not
// inside the bracket, or whose bracket values did not all fit (a wave's list
// part or the LDS stage), go to the exact fallback.  The list of column
// workgroup t is CAPB values: wave w's part from w * CAPW, nw[w] of them used.
template <int N>
__global__ __launch_bounds__(kSelThreads) void k_select(
    const ColPart *__restrict__ part, const float *__restrict__ list, int cbn,
    int nimg_w, int p0, int pbn, int npix, int dm_idx,
    int width_idx, int width, int64_t stat_base, rf_image_stats *__restrict__ stats,
    rf_candidate *__restrict__ cand, int ncap, int32_t *__restrict__ ncand,
    int32_t *__restrict__ fb_count, int32_t *__restrict__ fb_list, float thr, int t_begin,
    int t_end) {
  constexpr int CAPB = ColCfg<N>::COLS * N / 16;  // list values per column workgroup
  constexpr int NWC = ColCfg<N>::NT / 64;         // waves per column workgroup
  constexpr int CAPW = CAPB / NWC;                // list values per wave
  static_assert(CAPB % 64 == 0 && CAPW >= 16, "list parts");
  __shared__ uint32_t hist[kBins];
  __shared__ uint32_t wsum[kSelThreads / 64];
  __shared__ uint32_t sel[2];
  __shared__ float w_v[kSelThreads / 64];
  __shared__ int32_t w_i[kSelThreads / 64];
  __shared__ uint32_t w_lo[kSelThreads / 64];
  __shared__ uint32_t w_n[kSelThreads / 64];
  __shared__ uint32_t w_of[kSelThreads / 64];
  __shared__ float s_v;
  __shared__ int32_t s_i;
  __shared__ uint32_t s_lo, s_n, s_of;
  constexpr int CBN = N / ColCfg<N>::COLS;        // column workgroups per image
  constexpr int NV = lds_vals_of<N>();
  __shared__ uint32_t r_off[CBN * NWC];  // LDS offset of (workgroup, wave) values
  __shared__ uint32_t r_cnt[CBN * NWC];  // and their number
  __shared__ float vals[NV];
  __shared__ float binv[kBinCap];
  __shared__ uint32_t s_nc;
  __shared__ float s_med;
  const int il = blockIdx.x;
  const int pl = il >> 1;
  const int k = 2 * (p0 + pl) + (il & 1);
  if (pl >= pbn || k >= nimg_w) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const ColPart *pp = part + (size_t)il * cbn;
  {  // combine the column workgroups' records; workgroup r's values go to
     // LDS from r_off[r * NWC] (CBN / kSelThreads consecutive records per thread)
    constexpr int RPT = CBN > kSelThreads ? CBN / kSelThreads : 1;
    float v = -__builtin_inff();
    int32_t i = 0x7fffffff;
    uint32_t lo = 0, nn = 0, of = 0, cnt[RPT][NWC];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = RPT * tid + q;
#pragma unroll
      for (int w = 0; w < NWC; ++w) cnt[q][w] = 0;
      if (r < cbn) {
        const ColPart c = pp[r];
        if (better(c.maxv, c.maxi, v, i)) {
          v = c.maxv;
          i = c.maxi;
        }
        lo += c.cnt_lo;
#pragma unroll
        for (int w = 0; w < NWC; ++w) {
          cnt[q][w] = c.nw[w];
          nn += c.nw[w];
          of |= c.nw[w] > (uint32_t)CAPW;
        }
      }
    }
    uint32_t inc = nn;  // inclusive scan of the bracket counts over the block
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const float ov = __shfl_xor(v, o, 64);
      const int32_t oi = __shfl_xor(i, o, 64);
      if (better(ov, oi, v, i)) {
        v = ov;
        i = oi;
      }
      lo += __shfl_xor(lo, o, 64);
      of |= __shfl_xor(of, o, 64);
      const uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) w_n[wid] = inc;
    if (lane == 0) {
      w_v[wid] = v;
      w_i[wid] = i;
      w_lo[wid] = lo;
      w_of[wid] = of;
    }
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) {
      add += w < wid ? w_n[w] : 0u;
      tot += w_n[w];
    }
    uint32_t at = add + inc - nn;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = RPT * tid + q;
      if (r < cbn) {
#pragma unroll
        for (int w = 0; w < NWC; ++w) {
          r_off[r * NWC + w] = at;
          r_cnt[r * NWC + w] = min(cnt[q][w], (uint32_t)CAPW);
          at += cnt[q][w];
        }
      }
    }
    if (tid == 0) {
      for (int w = 1; w < kSelThreads / 64; ++w) {
        if (better(w_v[w], w_i[w], v, i)) {
          v = w_v[w];
          i = w_i[w];
        }
        lo += w_lo[w];
        of |= w_of[w];
      }
      s_v = v;
      s_i = i;
      s_lo = lo;
      s_n = tot;
      s_of = of;
    }
  }
  __syncthreads();
  const float peak = s_v;
  const int32_t pidx_ = s_i;
  const uint32_t rank = (uint32_t)(((size_t)npix * npix - 1) / 2);
  const uint32_t n = s_n;
  const bool ovf = s_of != 0 || n > (uint32_t)NV;
  float med;
  if (peak == 0.f && s_lo == 0 && n == 0) {
    med = 0.f;  // identically zero image (every pixel equals the zero peak)
  } else if (!ovf && s_lo <= rank && rank < s_lo + n) {
    uint32_t r = rank - s_lo;
    // Stage the kept magnitudes in LDS.  The list parts (one per wave of each
    // column workgroup, CAPW values apart) hold a few values each: 16 lanes
    // take one part, a wave four parts per load and 64 parts per round with
    // all 16 loads in flight; values past a part's sixteenth (rare) follow.
    const float *lr = list + (size_t)il * cbn * CAPB;
    constexpr int NWV = kSelThreads / 64;
    const int nparts = cbn * NWC, sub = lane >> 4, sl = lane & 15;
    for (int g0 = wid * 64; g0 < nparts; g0 += NWV * 64) {
      float x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int pt = min(g0 + 4 * u + sub, nparts - 1);
        x[u] = lr[(size_t)pt * CAPW + sl];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int pt = g0 + 4 * u + sub;
        if (pt < nparts) {
          const uint32_t c = r_cnt[pt], o = r_off[pt];
          if ((uint32_t)sl < c) vals[o + sl] = fabsf(x[u]);
          for (uint32_t e = 16 + sl; e < c; e += 16) vals[o + e] = fabsf(lr[(size_t)pt * CAPW + e]);
        }
      }
    }
    const float *lp = vals;
    // pass 1: 2048 equal-width bins over the bracket [lo, hi); the bin index
    // is a monotone function of the value, so the bin holding rank r holds
    // the wanted order statistic
    const float lo = pp[0].lo, hi = pp[0].hi;
    const float scale = (float)kBins / (hi - lo);
    for (int i = tid; i < kBins; i += kSelThreads) hist[i] = 0;
    if (tid == 0) s_nc = 0;
    __syncthreads();  // also: every staged value is in LDS
    for (uint32_t e = tid; e < n; e += kSelThreads)
      atomicAdd(&hist[min(kBins - 1, (int)((lp[e] - lo) * scale))], 1u);
    __syncthreads();
    sel_bin(hist, r, wsum, sel);
    const int b1 = (int)sel[0];
    const uint32_t r1 = sel[1];
    __syncthreads();
    // pass 2: gather that bin's values and rank them directly
    for (uint32_t e = tid; e < n; e += kSelThreads) {
      const float v = lp[e];
      if (min(kBins - 1, (int)((v - lo) * scale)) == b1) {
        const uint32_t at = atomicAdd(&s_nc, 1u);
        if (at < kBinCap) binv[at] = v;
      }
    }
    __syncthreads();
    const uint32_t nc = s_nc;
    if (nc <= kBinCap) {
      for (uint32_t t = tid; t < nc; t += kSelThreads) {
        const float v = binv[t];
        uint32_t less = 0, leq = 0;
        for (uint32_t u = 0; u < nc; ++u) {
          less += binv[u] < v;
          leq += binv[u] <= v;
        }
        if (less <= r1 && r1 < leq) s_med = v;  // equal values write the same value
      }
      __syncthreads();
      med = s_med;
    } else {
      // a crowded bin: exact three-pass radix select on the bit patterns
      // (bits 30..20, 19..9, 8..0)
      uint32_t prefix = 0;
      for (int pass = 0; pass < 3; ++pass) {
        for (int i = tid; i < kBins; i += kSelThreads) hist[i] = 0;
        __syncthreads();
        for (uint32_t e = tid; e < n; e += kSelThreads) {
          const uint32_t key = __float_as_uint(lp[e]);
          if (pass == 0) {
            atomicAdd(&hist[key >> 20], 1u);
          } else if (pass == 1) {
            if ((key >> 20) == prefix) atomicAdd(&hist[(key >> 9) & 2047u], 1u);
          } else {
            if ((key >> 9) == prefix) atomicAdd(&hist[key & 511u], 1u);
          }
        }
        __syncthreads();
        sel_bin(hist, r, wsum, sel);
        const uint32_t bin = sel[0];
        r = sel[1];
        __syncthreads();
        prefix = pass == 0 ? bin : (pass == 1 ? ((prefix << 11) | bin) : ((prefix << 9) | bin));
      }
      med = __uint_as_float(prefix);
    }
  } else {
    if (tid == 0) {
      const int slot = atomicAdd(fb_count, 1);
      fb_list[slot] = (int32_t)(stat_base + k);
    }
    return;
  }
  if (tid == 0) {
    const float sigma = 1.4826f * med;
    const float snr = sigma > 0.f ? peak / sigma : 0.f;
    const int x = pidx_ % npix, y = pidx_ / npix;
    if (stats) {
      rf_image_stats st;
      st.peak = peak;
      st.sigma = sigma;
      st.snr = snr;
      st.x = x;
      st.y = y;
      stats[stat_base + k] = st;
    }
    const int t_int = k * width;
    if (snr > thr && t_int >= t_begin && t_int < t_end) {
      const int slot = atomicAdd(ncand, 1);
      if (slot < ncap) {
        rf_candidate c;
        c.dm_idx = dm_idx;
        c.width_idx = width_idx;
        c.t_int = t_int;
        c.x = x;
        c.y = y;
        c.snr = snr;
        c.peak = peak;
        c.sigma = sigma;
        cand[slot] = c;
      }
    }
  }
}

// ------------------------------------------------------------------ host side
struct Shape {
  int pbw, cbp, pb, capb;  // capb: kept values per column workgroup (1/16 of its pixels)
};

template <int N>
Shape shape_n(const rf_plan *p) {
  Shape s;
  s.pbw = RowPairCfg<N>::PBW;
  s.cbp = N / ColCfg<N>::COLS;
  s.capb = ColCfg<N>::COLS * N / 16;
  static_assert(N / ColCfg<N>::COLS <= kMaxCB, "column workgroups per image");
  static_assert(ColCfg<N>::COLS * N / 16 >= 128, "a list region holds the staged 128 values");
  // pairs per batch: the row-transformed batches of all lanes (the plan's
  // budget, 240 MB by default) stay resident in the last-level cache between
  // the row and column passes
  const size_t per_pair = (size_t)std::max(1, p->n_rows) * N * sizeof(float2);
  const int pb = (int)std::max<size_t>(
      s.pbw, ((size_t)p->m_budget_mb << 20) / (size_t)p->lanes / per_pair);
  s.pb = std::min(64, (pb / s.pbw) * s.pbw);
  return s;
}

Shape shape_of(const rf_plan *p) {
  switch (p->npix) {
    case 64: return shape_n<64>(p);
    case 128: return shape_n<128>(p);
    case 256: return shape_n<256>(p);
    case 512: return shape_n<512>(p);
    case 1024: return shape_n<1024>(p);
    default: return shape_n<2048>(p);
  }
}

// Buffers of one lane (a stream that runs whole batches: cell sums, rows,
// columns and select, in order).
struct LaneBufs {
  size_t cv, m, epart, part, list;
};
// The dedispersed, resampled samples are double-buffered by DM parity, so
// that the next DM's pass over the segment overlaps this DM's batches.
struct Layout {
  size_t vi[2], fb, dd, rs, grid, img, mws, total;
  LaneBufs lane[kMaxLanes];
  std::vector<size_t> vi_off;  // per width, in float2 units
};

Layout layout_of(const rf_plan *p) {
  Layout L;
  const Shape sh = shape_of(p);
  const size_t nbc = (size_t)p->nbl * p->nchan;
  const size_t np2 = (size_t)p->npix * p->npix;
  size_t o = 0, vi_elems = 0;
  for (int j = 0; j < p->nwidth; ++j) {  // by image pair: [k / 2][bc][k % 2]
    L.vi_off.push_back(vi_elems);
    vi_elems += (size_t)((p->nint / p->width[j] + 1) / 2) * 2 * nbc;
  }
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  for (int d = 0; d < 2; ++d) L.vi[d] = take(vi_elems * sizeof(float2));
  for (int k = 0; k < p->lanes; ++k) {
    LaneBufs &b = L.lane[k];
    b.cv = take((size_t)2 * sh.pb * std::max(1, p->n_cells) * sizeof(float2));
    b.m = take((size_t)sh.pb * p->n_rows * p->npix * sizeof(float2));
    b.epart = take((size_t)sh.pb * std::max(1, p->n_rp) * 2 * sizeof(float));
    b.part = take((size_t)2 * sh.pb * sh.cbp * sizeof(ColPart));
    b.list = take((size_t)2 * sh.pb * sh.cbp * sh.capb * sizeof(float));
  }
  L.fb = take(((size_t)p->n_images + 1) * sizeof(int32_t));
  // buffers of the exact fallback (step chain on one image pair)
  const size_t sb = p->vis_dtype == RF_CF32 ? 8 : 4;
  L.dd = take((size_t)p->nint * nbc * p->npol * sb);
  L.rs = take((size_t)p->nint * nbc * p->npol * 8);
  L.grid = take(2 * np2 * 8);
  L.img = take(2 * np2 * 4);
  L.mws = take(image_ws_bytes(p, 2));
  L.total = o;
  return L;
}

// Optional event timing of every launch (rf_search_segment_profile): an
// event pair on the launch's own stream around each launch.  flush() waits for
// the recorded events (on every stream given to sync()) and sums the pairs.
struct Timer {
  rf_kernel_times *kt = nullptr;
  int sample = 1;  // time every sample-th launch of each kind (the first included)
  int64_t seen[RF_NK] = {};
  bool open = false;  // the launch between the current mark pair is timed
  std::vector<hipStream_t> streams;  // every stream that records events
  std::vector<hipEvent_t> pool;
  std::vector<int> kind;
  size_t used = 0;
  hipError_t mark(int k, hipStream_t s) {  // before (k >= 0) and after (k = -1) a launch
    if (!kt) return hipSuccess;
    if (k >= 0) {
      open = seen[k]++ % sample == 0;
      if (!open) return hipSuccess;
    } else {
      if (!open) return hipSuccess;
      open = false;
    }
    if (used == pool.size()) {
      hipEvent_t e;
      const hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return err;
      pool.push_back(e);
    }
    if (k >= 0) kind.push_back(k);
    return hipEventRecord(pool[used++], s);
  }
  // Launches kernel k of `kind` on s.  A sampled launch carries a start and a
  // stop event recorded by the dispatch itself (hipExtLaunchKernel): no
  // packets are added to the stream around it, so the schedule is the
  // untimed one and the duration is the kernel's own.
  template <typename... KArgs, typename... Args>
  hipError_t launch(int k, void (*kern)(KArgs...), dim3 grid, dim3 block, hipStream_t s,
                    Args... args) {
    static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kt && seen[k]++ % sample == 0) {
      while (pool.size() < used + 2) {
        hipEvent_t e;
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        pool.push_back(e);
      }
      e0 = pool[used];
      e1 = pool[used + 1];
      used += 2;
      kind.push_back(k);
    }
    if (e0) {
      hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0u, static_cast<KArgs>(args)...);
    } else {
      // untimed launches (every launch of rf_search_segment and of a batch,
      // captured or not) use the plain launch, which stream capture records
      // as a kernel node; the extension launch is kept to timed profiles
      hipLaunchKernelGGL(kern, grid, block, 0, s, static_cast<KArgs>(args)...);
    }
    return hipGetLastError();
  }
  bool full() const { return used >= 32768; }
  hipError_t flush() {
    if (!kt || used == 0) return hipSuccess;
    for (hipStream_t s : streams) {
      const hipError_t err = hipStreamSynchronize(s);
      if (err != hipSuccess) return err;
    }
    for (size_t q = 0; q + 1 < used; q += 2) {
      float ms = 0.f;
      const hipError_t err = hipEventElapsedTime(&ms, pool[q], pool[q + 1]);
      if (err != hipSuccess) return err;
      kt->ms[kind[q / 2]] += ms;
      kt->launches[kind[q / 2]] += 1;
    }
    used = 0;
    kind.clear();
    return hipSuccess;
  }
  ~Timer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// Streams and events of a segment search: lane streams, a stream for the
// per-DM pass over the segment, and the events ordering them; default
// priority.  Created per call, or once per batch (kept until the batch's
// graph is destroyed).
struct Lanes {
  hipStream_t lane[kMaxLanes] = {}, drs = nullptr;
  hipEvent_t start = nullptr, drs_done[2] = {}, lane_dm[kMaxLanes][2] = {},
             lane_end[kMaxLanes] = {}, drs_end = nullptr;
  // nl lane streams and the pass stream: only the streams a search uses, so
  // that with the caller's stream they fit the device's hardware queues
  // without two of them sharing one
  hipError_t init(int nl) {
    hipError_t e = hipStreamCreateWithFlags(&drs, hipStreamNonBlocking);
    for (int k = 0; k < std::min(nl, kMaxLanes) && e == hipSuccess; ++k)
      e = hipStreamCreateWithFlags(&lane[k], hipStreamNonBlocking);
    auto ev = [&](hipEvent_t &x) {
      if (e == hipSuccess) e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
    };
    ev(start);
    ev(drs_end);
    for (int d = 0; d < 2; ++d) ev(drs_done[d]);
    for (int k = 0; k < kMaxLanes; ++k) {
      ev(lane_dm[k][0]);
      ev(lane_dm[k][1]);
      ev(lane_end[k]);
    }
    return e;
  }
  ~Lanes() {
    // a search that returned early (an error part way) can leave work on the
    // lane streams that the caller's stream never joined: let it finish
    // before the caller reuses the buffers (instant on the normal path)
    for (int k = 0; k < kMaxLanes; ++k)
      if (lane[k]) (void)hipStreamSynchronize(lane[k]);
    if (drs) (void)hipStreamSynchronize(drs);
    auto de = [](hipEvent_t x) {
      if (x) (void)hipEventDestroy(x);
    };
    de(start);
    de(drs_end);
    for (int d = 0; d < 2; ++d) de(drs_done[d]);
    for (int k = 0; k < kMaxLanes; ++k) {
      de(lane_dm[k][0]);
      de(lane_dm[k][1]);
      de(lane_end[k]);
      if (lane[k]) (void)hipStreamDestroy(lane[k]);
    }
    if (drs) (void)hipStreamDestroy(drs);
  }
};

// One batch (pbn image pairs from p0 of one (DM, width)), every launch on
// stream s with the lane's buffers.
template <int N>
rf_status batch_n(const rf_plan *p, const Shape &sh, const float2 *vi, int nimg_w, int p0,
                  int pbn, int dm_idx, int width_idx, int width, int64_t stat_base, char *ws,
                  const LaneBufs &B, int32_t *fb, rf_image_stats *stats, rf_candidate *cand,
                  int cap, int32_t *ncand, hipStream_t s, Timer *tm) {
  float2 *M = (float2 *)(ws + B.m);
  float4 *cv = (float4 *)(ws + B.cv);
  float *epart = (float *)(ws + B.epart);
  ColPart *part = (ColPart *)(ws + B.part);
  float *list = (float *)(ws + B.list);
  const int npb = (pbn + sh.pbw - 1) / sh.pbw;
  const int nimg_b = std::min(2 * pbn, nimg_w - 2 * p0);  // images in this batch
  // groups of kCellPairs image pairs; with fewer than eight, several XCDs
  // share each group's cell blocks so that no XCD idles
  const int npair = (nimg_b + 1) / 2;
  const int ngrp = (npair + kCellPairs - 1) / kCellPairs;
  const int rep = ngrp >= 8 ? 1 : 8 / ngrp;
  const int per_xcd = rep == 1 ? (ngrp + 7) / 8 * p->n_cblk : (p->n_cblk + rep - 1) / rep;
  RF_HIP_TRY(tm->launch(RF_K_GRID, k_cellsum, dim3(8 * per_xcd), dim3(kCellThreads), s,
                        (const float4 *)vi, p->nbl * p->nchan, p0, npair, p->n_cells,
                        p->n_cblk, p->d_cblk, p->d_ucell_off, p->d_contrib, cv, rep));
  RF_HIP_TRY(tm->launch(RF_K_ROWS, k_rows_pairs<N>, dim3(npb * p->n_rp), dim3(RowPairCfg<N>::NT),
                        s, cv, p->n_cells, nimg_w, p0, pbn, p->d_rp_row, p->d_rp_sa, p->d_rp_sb,
                        p->n_rp, p->n_rows, p->d_zs_off, p->d_zs_u, p->d_zs_ck, p->d_zs_cmk,
                        half_inv_w(p), p->d_tw, M, epart));
  const float inv_w = 1.0f / (float)p->W;
  const int cgrid = (pbn * sh.cbp + 7) / 8 * 8;
  RF_HIP_TRY(tm->launch(RF_K_COLS, k_cols_stats<N>, dim3(cgrid), dim3(ColCfg<N>::NT), s, M,
                        p->n_rows, p->vmax, nimg_w, p0, pbn, inv_w, p->d_tw, epart, p->n_rp, part,
                        list, sh.capb));
  RF_HIP_TRY(tm->launch(RF_K_SELECT, k_select<N>, dim3(2 * pbn), dim3(kSelThreads), s, part,
                        list, sh.cbp, nimg_w, p0, pbn, N, dm_idx, width_idx, width, stat_base,
                        stats, cand, cap, ncand, fb, fb + 1, p->threshold, p->t_begin,
                        p->t_end));
  return RF_OK;
}

rf_status batch(const rf_plan *p, const Shape &sh, const float2 *vi, int nimg_w, int p0, int pbn,
                int dm_idx, int width_idx, int width, int64_t stat_base, char *ws,
                const LaneBufs &B, int32_t *fb, rf_image_stats *stats, rf_candidate *cand,
                int cap, int32_t *ncand, hipStream_t s, Timer *tm) {
#define RF_BATCH(NN)                                                                            \
  return batch_n<NN>(p, sh, vi, nimg_w, p0, pbn, dm_idx, width_idx, width, stat_base, ws, B, \
                     fb, stats, cand, cap, ncand, s, tm)
  switch (p->npix) {
    case 64: RF_BATCH(64);
    case 128: RF_BATCH(128);
    case 256: RF_BATCH(256);
    case 512: RF_BATCH(512);
    case 1024: RF_BATCH(1024);
    default: RF_BATCH(2048);
  }
#undef RF_BATCH
}

int lcm_int(int a, int b) { return a / std::gcd(a, b) * b; }

}  // namespace

namespace {
rf_status drs_timed(const rf_plan *p, const int32_t *d_delay_row, const void *vis,
                    const int *widths, int nw, float2 *const *vi_out, hipStream_t s, Timer *tm) {
  const int nbc = p->nbl * p->nchan;
  // process the widths in groups of kMaxW whose least common multiple keeps a
  // time chunk short; each group reads the segment once
  int j = 0;
  while (j < nw) {
    WidthSet ws{};
    int L = 1, n = 0;
    while (j + n < nw && n < kMaxW) {
      const int L2 = lcm_int(L, widths[j + n]);
      if (n > 0 && L2 > 256) break;
      L = L2;
      ws.w[n] = widths[j + n];
      ws.nk[n] = p->nint / widths[j + n];
      ws.out[n] = vi_out[j + n];
      ++n;
    }
    ws.nw = n;
    // 16 integrations per thread (or the multiple of the widths' least common
    // multiple that holds an even number of images of every width): measured
    // 1170 us per survey DM trial against 1177 us at 8, 1192 at 24, 1212 at
    // 32 and 1229 at 64 (with 256 threads and 8 loads in flight per thread;
    // 128 or 512 threads, 4, 12 or 16 loads in flight were slower)
    const int tchunk = L * std::max(2, (16 / L + 1) & ~1);
    dim3 grid((nbc + kDrsThreads - 1) / kDrsThreads, (p->nint + tchunk - 1) / tchunk);
    const dim3 blk(kDrsThreads);
    if (p->vis_dtype == RF_CF32) {
      if (p->npol == 2)
        RF_HIP_TRY(tm->launch(RF_K_DRS, k_drs<float2, 2>, grid, blk, s, (const float2 *)vis,
                              d_delay_row, p->nint, nbc, p->nchan, tchunk, ws));
      else
        RF_HIP_TRY(tm->launch(RF_K_DRS, k_drs<float2, 1>, grid, blk, s, (const float2 *)vis,
                              d_delay_row, p->nint, nbc, p->nchan, tchunk, ws));
    } else {
      if (p->npol == 2)
        RF_HIP_TRY(tm->launch(RF_K_DRS, k_drs<__half2, 2>, grid, blk, s, (const __half2 *)vis,
                              d_delay_row, p->nint, nbc, p->nchan, tchunk, ws));
      else
        RF_HIP_TRY(tm->launch(RF_K_DRS, k_drs<__half2, 1>, grid, blk, s, (const __half2 *)vis,
                              d_delay_row, p->nint, nbc, p->nchan, tchunk, ws));
    }
    j += n;
  }
  return RF_OK;
}
}  // namespace

size_t segment_ws_bytes(const rf_plan *p) {
  if (p->W == 0 || p->n_rows == 0) return std::max(layout_of(p).total, steps_ws_bytes(p));
  return layout_of(p).total;
}

// Enqueues the fused search of one segment on stream s and the lane streams
// of `lanes` (joined to s at the end): no host synchronisation, so a batch can
// capture it into a graph.  The images whose median left the bracket are
// listed in fb ([0] = count, then global image indices) for segment_finish.
// serial: every launch in order on s (timed kernels that do not overlap).
//
// DM trials dm0 .. dm1 - 1 only (a segment may be enqueued in several DM
// ranges, in order, on one stream: the first range clears the counters; a
// range does not wait on the events of an earlier one, whose work the stream
// order already puts first).
rf_status segment_enqueue(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                          int32_t *ncand, rf_image_stats *stats, char *ws, size_t ws_bytes,
                          int32_t *fb, hipStream_t s, Lanes *lanes, bool serial, Timer *tm,
                          int dm0 = 0, int dm1 = -1) {
  const Layout L = layout_of(p);
  const Shape sh = shape_of(p);
  if (dm1 < 0) dm1 = p->ndm;
  rf_status st = RF_OK;
  if (dm0 == 0) {
    st = launch_zero_i32(ncand, 1, s);
    if (st != RF_OK) return st;
    st = launch_zero_i32(fb, 1, s);
    if (st != RF_OK) return st;
  }
  if (p->W == 0 || p->n_rows == 0) {
    if (dm0 > 0) return RF_OK;  // the first range did the whole segment
    // nothing is gridded: every image is identically zero; the step chain
    // produces the (zero) statistics.  Its buffers start at the workspace's
    // first byte and can cover the fallback list, so the count is cleared
    // again after it (stream order): no image needs the exact recomputation.
    st = run_segment_steps(p, vis, cand, cap, ncand, stats, ws, ws_bytes, s);
    if (st != RF_OK) return st;
    return launch_zero_i32(fb, 1, s);
  }
  // The lane streams take the batches round robin and a stream of its own
  // runs each DM's pass over the segment into the sample buffer of that DM's
  // parity.  The pass of DM i waits until every lane has finished the batches
  // of DM i - 2 (the last readers of that buffer); a lane's batches of DM i
  // wait for the pass of DM i.
  const int nl = serial ? 1 : p->lanes;
  hipStream_t ls[kMaxLanes], ds = s;
  for (int k = 0; k < kMaxLanes; ++k) ls[k] = s;
  if (!serial) {
    RF_HIP_TRY(hipEventRecord(lanes->start, s));
    RF_HIP_TRY(hipStreamWaitEvent(lanes->drs, lanes->start, 0));
    ds = lanes->drs;
    for (int k = 0; k < nl; ++k) {
      ls[k] = lanes->lane[k];
      RF_HIP_TRY(hipStreamWaitEvent(ls[k], lanes->start, 0));
    }
    // the caller's stream stays in the list: the exact fallback records there
    tm->streams.insert(tm->streams.end(), ls, ls + nl);
    tm->streams.push_back(ds);
  }
  int nbatch = 0;
  std::vector<float2 *> vi_out(p->nwidth);
  auto samples_of = [&](int i) {  // the sample buffer of DM i's parity, per width
    float2 *vi = (float2 *)(ws + L.vi[i & 1]);
    for (int j = 0; j < p->nwidth; ++j) vi_out[j] = vi + L.vi_off[j];
  };
  // The pass of DM i is enqueued as early as its buffer allows, right after
  // the batches of DM i - 2 (its last readers), so that it can run while the
  // batches of DM i - 1 do: the host enqueues a DM's batches at about the
  // rate the device runs them, and a pass enqueued just before the batches of
  // its own DM reached the device only when the lanes were about to wait for
  // it.  (Running beside the batches, the pass and the batches each slow
  // down by about the other's share: the search takes the same time either
  // way, but no longer depends on the host keeping ahead.)
  auto enqueue_pass = [&](int i) -> rf_status {
    samples_of(i);
    if (!serial && i - 2 >= dm0)
      for (int k = 0; k < nl; ++k) RF_HIP_TRY(hipStreamWaitEvent(ds, lanes->lane_dm[k][i & 1], 0));
    const rf_status r = drs_timed(p, p->d_delay + (size_t)i * p->nchan, vis, p->width.data(),
                                  p->nwidth, vi_out.data(), ds, tm);
    if (r != RF_OK) return r;
    if (!serial) RF_HIP_TRY(hipEventRecord(lanes->drs_done[i & 1], ds));
    return RF_OK;
  };
  for (int i = dm0; i < std::min(dm1, dm0 + 2); ++i) {
    st = enqueue_pass(i);
    if (st != RF_OK) return st;
  }
  for (int i = dm0; i < dm1; ++i) {
    samples_of(i);
    if (!serial)  // the latest record of drs_done[i & 1] is DM i's pass
      for (int k = 0; k < nl; ++k)
        RF_HIP_TRY(hipStreamWaitEvent(ls[k], lanes->drs_done[i & 1], 0));
    for (int j = 0; j < p->nwidth; ++j) {
      const int w = p->width[j];
      const int nimg_w = p->nint / w;
      const int npairs = (nimg_w + 1) / 2;
      const int64_t base = p->img_base[(size_t)i * p->nwidth + j];
      for (int p0 = 0; p0 < npairs; p0 += sh.pb) {
        const int pbn = std::min(sh.pb, npairs - p0);
        const int k = nbatch % nl;
        st = batch(p, sh, vi_out[j], nimg_w, p0, pbn, i, j, w, base, ws, L.lane[k], fb, stats,
                   cand, cap, ncand, ls[k], tm);
        if (st != RF_OK) return st;
        ++nbatch;
      }
    }
    if (!serial)
      for (int k = 0; k < nl; ++k) RF_HIP_TRY(hipEventRecord(lanes->lane_dm[k][i & 1], ls[k]));
    if (i + 2 < dm1) {
      st = enqueue_pass(i + 2);
      if (st != RF_OK) return st;
    }
    // timed serially: flush every DM; timed concurrently: only when the event
    // pool is large (a flush drains the lanes)
    if (tm->kt && (serial || tm->full())) RF_HIP_TRY(tm->flush());
  }
  if (!serial) {  // join: the caller's stream waits for every lane and the pass stream
    for (int k = 0; k < nl; ++k) {
      RF_HIP_TRY(hipEventRecord(lanes->lane_end[k], ls[k]));
      RF_HIP_TRY(hipStreamWaitEvent(s, lanes->lane_end[k], 0));
    }
    // the last pass is already ordered before the lanes' last batches; the
    // explicit join makes every stream forked from s end in s, which stream
    // capture requires of each forked stream
    RF_HIP_TRY(hipEventRecord(lanes->drs_end, ds));
    RF_HIP_TRY(hipStreamWaitEvent(s, lanes->drs_end, 0));
  }
  return RF_OK;
}

// Exact fallback of the images listed in fb: reads the list (one host
// synchronisation of s) and recomputes each listed image with the step chain
// (paired with its partner image, for identical rounding), replacing its
// statistics and adding its candidate.
rf_status segment_finish(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                         int32_t *ncand, rf_image_stats *stats, char *ws, const int32_t *fb,
                         hipStream_t s, Timer *tm) {
  const Layout L = layout_of(p);
  const size_t nbc = (size_t)p->nbl * p->nchan;
  rf_status st = RF_OK;
  int32_t nfb = 0;
  RF_HIP_TRY(hipMemcpyAsync(&nfb, fb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  RF_HIP_TRY(hipStreamSynchronize(s));
  if (nfb == 0) return RF_OK;
  std::vector<int32_t> idx(nfb);
  RF_HIP_TRY(hipMemcpyAsync(idx.data(), fb + 1, sizeof(int32_t) * nfb, hipMemcpyDeviceToHost, s));
  RF_HIP_TRY(hipStreamSynchronize(s));
  std::sort(idx.begin(), idx.end());
  void *dd = ws + L.dd;
  float2 *rs = (float2 *)(ws + L.rs);
  float2 *grid = (float2 *)(ws + L.grid);
  float *img = (float *)(ws + L.img);
  float2 *mws = (float2 *)(ws + L.mws);
  const size_t per_int = nbc * p->npol;
  int cur_i = -1, cur_j = -1;
  for (int32_t g : idx) {
    // image index -> (dm, width, k)
    int i = 0, j = 0;
    for (i = p->ndm - 1; i > 0 && p->img_base[(size_t)i * p->nwidth] > g; --i) {
    }
    for (j = p->nwidth - 1; j > 0 && p->img_base[(size_t)i * p->nwidth + j] > g; --j) {
    }
    const int k = (int)(g - p->img_base[(size_t)i * p->nwidth + j]);
    const int w = p->width[j];
    if (i != cur_i) {
      st = launch_dedisperse(p, p->d_delay + (size_t)i * p->nchan, vis, dd, s);
      if (st != RF_OK) return st;
      cur_i = i;
      cur_j = -1;
    }
    if (j != cur_j) {
      st = launch_resample(p, w, dd, p->vis_dtype, p->nint, rs, s);
      if (st != RF_OK) return st;
      cur_j = j;
    }
    RF_HIP_TRY(tm->mark(RF_K_FALLBACK, s));
    const int k0 = k & ~1;
    const int npair = std::min(2, p->nint / w - k0);
    st = launch_grid_dense(p, rs + (size_t)k0 * per_int, npair, grid, s);
    if (st != RF_OK) return st;
    st = launch_image_dense(p, grid, npair, img, mws, s);
    if (st != RF_OK) return st;
    const rf_tag_gen gen{i, j, w, k};
    st = launch_search(p, img + (size_t)(k - k0) * p->npix * p->npix, 1, nullptr, &gen,
                       stats ? stats + g : nullptr, cand, cap, ncand, s);
    if (st != RF_OK) return st;
    RF_HIP_TRY(tm->mark(-1, s));
  }
  return RF_OK;
}

rf_status run_segment(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                      int32_t *ncand, rf_image_stats *stats, void *ws_v, size_t ws_bytes,
                      hipStream_t s, rf_kernel_times *kt) {
  Timer timer;
  timer.kt = kt;
  if (kt) timer.sample = std::max(1, kt->sample);
  timer.streams.push_back(s);
  char *ws = static_cast<char *>(ws_v);
  int32_t *fb = (int32_t *)(ws + layout_of(p).fb);
  const bool serial = kt && !kt->concurrent;
  Lanes lanes;
  if (!serial) RF_HIP_TRY(lanes.init(p->lanes));
  rf_status st =
      segment_enqueue(p, vis, cand, cap, ncand, stats, ws, ws_bytes, fb, s, &lanes, serial, &timer);
  if (st != RF_OK) return st;
  RF_HIP_TRY(timer.flush());
  st = segment_finish(p, vis, cand, cap, ncand, stats, ws, fb, s, &timer);
  if (st != RF_OK) return st;
  RF_HIP_TRY(timer.flush());
  return RF_OK;
}

// A segment search split in two: begin enqueues everything but the exact
// fallback and returns at once; end waits for the fallback list, recomputes
// the listed images and frees the job (its lane streams live until then).
struct rf_segment_job {
  const rf_plan *p;
  const void *vis;
  rf_candidate *cand;
  int cap;
  int32_t *ncand;
  rf_image_stats *stats;
  char *ws;
  int32_t *fb;
  hipStream_t s;
  Lanes lanes;
};

rf_status segment_begin(const rf_plan *p, const void *vis, rf_candidate *cand, int cap,
                        int32_t *ncand, rf_image_stats *stats, void *ws_v, size_t ws_bytes,
                        hipStream_t s, rf_segment_job **out) {
  rf_segment_job *j = new rf_segment_job();
  j->p = p;
  j->vis = vis;
  j->cand = cand;
  j->cap = cap;
  j->ncand = ncand;
  j->stats = stats;
  j->ws = static_cast<char *>(ws_v);
  j->fb = (int32_t *)(j->ws + layout_of(p).fb);
  j->s = s;
  if (j->lanes.init(p->lanes) != hipSuccess) {
    delete j;
    return RF_EHIP;
  }
  Timer none;
  none.streams.push_back(s);
  const rf_status st = segment_enqueue(p, vis, cand, cap, ncand, stats, j->ws, ws_bytes, j->fb, s,
                                       &j->lanes, false, &none);
  if (st != RF_OK) {
    delete j;  // drains the lane streams
    return st;
  }
  *out = j;
  return RF_OK;
}

rf_status segment_end(rf_segment_job *j) {
  Timer none;
  none.streams.push_back(j->s);
  const rf_status st =
      segment_finish(j->p, j->vis, j->cand, j->cap, j->ncand, j->stats, j->ws, j->fb, j->s, &none);
  delete j;
  return st;
}

// ------------------------------------------------------------------ batches
// A batch searches several segments (plans of any shapes) bound once: the
// segments run in order, sharing one workspace, each with its own fallback
// list.  rf_batch_run runs every segment's fused search, then the exact
// fallbacks.
//
// With RF_BATCH_GRAPH the enqueue of every segment is captured once, at
// create, into one HIP graph and each run is one graph launch.  The capture
// runs on a stream of the batch's own (never the caller's, which may be the
// null stream, where capture is not allowed), in thread-local mode, and
// records only kernel launches (plain launches: the zeroing of counters is a
// kernel too, no memset node) and the event joins of the lane and pass
// streams forked from the capture stream, every one of which is joined back
// before the capture ends.
struct rf_batch {
  std::vector<const rf_plan *> plans;
  std::vector<const void *> vis;
  std::vector<rf_candidate *> cand;
  std::vector<int32_t> cap;
  std::vector<int32_t *> ncand;
  std::vector<rf_image_stats *> stats;
  std::vector<int32_t *> fb;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  Lanes lanes;
  hipStream_t cap_stream = nullptr;  // capture stream (graph mode)
  std::vector<hipGraph_t> graphs;     // the batch's work, in launch order
  std::vector<hipGraphExec_t> execs;
  size_t graph_nodes = 0;
  ~rf_batch() {
    for (hipGraphExec_t x : execs) (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : graphs) (void)hipGraphDestroy(g);
    if (cap_stream) {
      (void)hipStreamSynchronize(cap_stream);
      (void)hipStreamDestroy(cap_stream);
    }
  }
};

size_t batch_ws_bytes(const rf_plan *const *plans, int nseg, size_t *main_bytes) {
  size_t m = 0, f = 0;
  for (int i = 0; i < nseg; ++i) {
    m = std::max(m, segment_ws_bytes(plans[i]));
    f += align_up(((size_t)plans[i]->n_images + 1) * sizeof(int32_t));
  }
  if (main_bytes) *main_bytes = align_up(m);
  return align_up(m) + f;
}

namespace {
// Kernel launches one DM trial of the fused search enqueues.
size_t launches_per_dm(const rf_plan *p) {
  if (p->W == 0 || p->n_rows == 0) return 1;
  const Shape sh = shape_of(p);
  size_t n = (size_t)p->nwidth;  // passes over the segment (at most one per width)
  for (int j = 0; j < p->nwidth; ++j) {
    const int npairs = (p->nint / p->width[j] + 1) / 2;
    n += 4 * (size_t)((npairs + sh.pb - 1) / sh.pb);
  }
  return n;
}

rf_status batch_enqueue_all(rf_batch *b, hipStream_t s) {
  Timer none;
  none.streams.push_back(s);
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const rf_status st =
        segment_enqueue(b->plans[i], b->vis[i], b->cand[i], b->cap[i], b->ncand[i], b->stats[i],
                        b->ws, b->ws_bytes, b->fb[i], s, &b->lanes, false, &none);
    if (st != RF_OK) return st;
  }
  return RF_OK;
}

// One captured graph: the DM trials [dm0, dm1) of each listed segment.
struct GraphPart {
  std::vector<int> seg, dm0, dm1;
};

rf_status capture_part(rf_batch *b, const GraphPart &gp) {
  RF_HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  Timer none;
  none.streams.push_back(b->cap_stream);
  rf_status st = RF_OK;
  for (size_t q = 0; q < gp.seg.size() && st == RF_OK; ++q) {
    const int i = gp.seg[q];
    st = segment_enqueue(b->plans[i], b->vis[i], b->cand[i], b->cap[i], b->ncand[i], b->stats[i],
                         b->ws, b->ws_bytes, b->fb[i], b->cap_stream, &b->lanes, false, &none,
                         gp.dm0[q], gp.dm1[q]);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);  // ends the capture in any case
  if (st != RF_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return st != RF_OK ? st : RF_EHIP;
  }
  b->graphs.push_back(g);
  size_t n = 0;
  RF_HIP_TRY(hipGraphGetNodes(g, nullptr, &n));
  b->graph_nodes += n;
  hipGraphExec_t x = nullptr;
  RF_HIP_TRY(hipGraphInstantiate(&x, g, nullptr, nullptr, 0));
  b->execs.push_back(x);
  return RF_OK;
}

// The batch's work split into graphs of at most kGraphLaunches kernel
// launches (whole DM trials; a DM trial of more launches forms a graph of its
// own), captured in order.  Each graph forks the lane streams from the
// capture stream and joins them back; graphs run one after another on the
// caller's stream.
constexpr size_t kGraphLaunches = 8192;

[[maybe_unused]] rf_status batch_capture(rf_batch *b) {
  RF_HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  GraphPart cur;
  size_t used = 0;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const rf_plan *p = b->plans[i];
    const size_t per = launches_per_dm(p);
    int d = 0;
    while (d < p->ndm) {
      // W = 0: the whole segment is one step-chain range
      const int take = (p->W == 0 || p->n_rows == 0)
                           ? p->ndm
                           : (int)std::min<size_t>(p->ndm - d,
                                                   std::max<size_t>(1, (kGraphLaunches - std::min(used, kGraphLaunches)) / per));
      if (used > 0 && used + per > kGraphLaunches) {
        const rf_status st = capture_part(b, cur);
        if (st != RF_OK) return st;
        cur = GraphPart();
        used = 0;
        continue;
      }
      cur.seg.push_back((int)i);
      cur.dm0.push_back(d);
      cur.dm1.push_back(d + take);
      used += per * (size_t)take;
      d += take;
    }
  }
  if (!cur.seg.empty()) return capture_part(b, cur);
  return RF_OK;
}
}  // namespace

rf_status batch_create(const rf_plan *const *plans, int nseg, const void *const *d_vis,
                       rf_candidate *const *d_cand, const int32_t *cap, int32_t *const *d_ncand,
                       rf_image_stats *const *d_stats, void *d_ws, size_t ws_bytes, int flags,
                       rf_batch **out) {
  size_t main_bytes = 0;
  if (ws_bytes < batch_ws_bytes(plans, nseg, &main_bytes)) return RF_EWORKSPACE;
  rf_batch *b = new rf_batch();
  b->ws = (char *)d_ws;
  b->ws_bytes = main_bytes;
  size_t off = main_bytes;
  for (int i = 0; i < nseg; ++i) {
    b->plans.push_back(plans[i]);
    b->vis.push_back(d_vis[i]);
    b->cand.push_back(d_cand[i]);
    b->cap.push_back(cap[i]);
    b->ncand.push_back(d_ncand[i]);
    b->stats.push_back(d_stats ? d_stats[i] : nullptr);
    b->fb.push_back((int32_t *)(b->ws + off));
    off += align_up(((size_t)plans[i]->n_images + 1) * sizeof(int32_t));
  }
  int max_lanes = 1;
  for (int i = 0; i < nseg; ++i) max_lanes = std::max(max_lanes, (int)plans[i]->lanes);
  if (b->lanes.init(max_lanes) != hipSuccess) {
    delete b;
    return RF_EHIP;
  }
  if (flags & RF_BATCH_GRAPH) {
    // Switched off: both runs of a captured batch (the first with the
    // caller's stream as capture origin and extension launches, the second
    // as above: the batch's own stream, plain launches, every forked stream
    // joined, graphs of at most kGraphLaunches launches) ended the host
    // process with a segmentation fault inside rf_batch_create, for a batch of
    // four small segments whose eager run is correct.  Reading this capture
    // sequence found every call documented as capturable; until a cause is
    // shown the request is refused rather than run.
    delete b;
    return RF_EUNSUPPORTED;
  }
  *out = b;
  return RF_OK;
}

rf_status batch_run(rf_batch *b, hipStream_t s) {
  if (!b->execs.empty()) {
    for (hipGraphExec_t x : b->execs) RF_HIP_TRY(hipGraphLaunch(x, s));
  } else {
    const rf_status st = batch_enqueue_all(b, s);
    if (st != RF_OK) return st;
  }
  Timer none;
  none.streams.push_back(s);
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const rf_status st = segment_finish(b->plans[i], b->vis[i], b->cand[i], b->cap[i], b->ncand[i],
                                        b->stats[i], b->ws, b->fb[i], s, &none);
    if (st != RF_OK) return st;
  }
  return RF_OK;
}

size_t batch_graph_nodes(const rf_batch *b) { return b->graph_nodes; }

void batch_destroy(rf_batch *b) { delete b; }
