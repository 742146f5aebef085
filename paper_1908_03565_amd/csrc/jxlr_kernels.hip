// HIP kernels of the VarDCT reconstruction library for CDNA4 (gfx950), and
// the C-ABI entry points that launch them.
//
// Kernels (all 256 threads = 4 wave64 per workgroup):
//   recon_kernel   one workgroup per 32x32-pixel region: F.2/F.3 dequant,
//                  Annex G chroma from luma, I.2.7 LLF from DC and the I.2.4
//                  inverse transforms, staged in LDS; writes XYB planes.
//   epf_kernel     one workgroup per 32x32 output tile: one J.2 pass with the
//                  tile and its filter halo staged in LDS.
//   finish_kernel  one thread per pixel: J.4 Gaborish and L.2 XYB -> RGB,
//                  optional sRGB 8/16-bit encoding.
// Varblocks are naturally aligned and at most 32x32 (C.5.4), so every
// varblock lies inside exactly one 32x32 region; the region is the unit of
// work of the reconstruction and of the EPF sigma computation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/jxlr.h"
#include "jxlr_tables.h"

using jxlr::DeviceTables;

struct jxlr_ctx {
  int device;
  DeviceTables* tables;  // device memory
  int* status;           // device memory, sticky validation flag
};

namespace {

constexpr int kThreads = 256;
constexpr uint8_t kAbsent = 0xFF;

// Varblock size in blocks of transform type s (I.2.5): "DCT N x M" is N wide.
__host__ __device__ constexpr int vb_bx(int s) {
  return (s == 4 || s == 6 || s == 11) ? 2 : (s == 5 || s == 8 || s == 10) ? 4 : 1;
}
__host__ __device__ constexpr int vb_by(int s) {
  return (s == 4 || s == 7 || s == 10) ? 2 : (s == 5 || s == 9 || s == 11) ? 4 : 1;
}
// Offset of type s inside DeviceTables::dq.
__host__ __device__ constexpr int dq_off(int s) {
  int off = 0;
  for (int t = 0; t < s; ++t) off += 192 * vb_bx(t) * vb_by(t);
  return off;
}
static_assert(dq_off(jxlr::kNumStrategies) == jxlr::kDqFloats, "dequant table layout");

__device__ inline int mirror(int c, int size) {
  // 6.5: reflect with the edge sample repeated, as often as needed
  while (c < 0 || c >= size) c = c < 0 ? -c - 1 : 2 * size - 1 - c;
  return c;
}

// Raster scan of the blocks of one region (C.5.4).  nbx, nby: blocks of the
// region inside the frame.  raw: DctSelect values; owner/strat: per block the
// index of its varblock's top-left block and the type, kAbsent outside.
__device__ bool scan_region(const uint8_t* raw, int nbx, int nby, uint8_t* owner,
                            uint8_t* strat) {
  for (int i = 0; i < 16; ++i) owner[i] = strat[i] = kAbsent;
  for (int by = 0; by < nby; ++by)
    for (int bx = 0; bx < nbx; ++bx) {
      const int i = by * 4 + bx;
      if (owner[i] != kAbsent) continue;
      const int s = raw[i];
      if (s >= jxlr::kNumStrategies) return false;
      const int cx = vb_bx(s), cy = vb_by(s);
      // regions start at multiples of 4 blocks, so local alignment is global
      if ((bx % cx) || (by % cy) || bx + cx > nbx || by + cy > nby) return false;
      for (int j = 0; j < cy; ++j)
        for (int k = 0; k < cx; ++k) {
          const int m = (by + j) * 4 + bx + k;
          if (owner[m] != kAbsent) return false;
          owner[m] = uint8_t(i);
          strat[m] = uint8_t(s);
        }
    }
  return true;
}

struct ReconArgs {
  int W, H, Wb, Hb;
  const int32_t* ac[3];
  size_t ac_stride;
  const int32_t* dc[3];
  size_t dc_stride;
  const uint8_t* strategy;
  const uint8_t* qf;
  size_t map_stride;
  const float* cfl_kx;
  const float* cfl_kb;
  size_t cfl_stride;
  float dc_mul[3];  // already divided by 2^extra_levels
  float kx_dc, kb_dc;
  float gscale;     // global_scale as float (exact)
  float one_bias[3];
  float* xyb;
  size_t xyb_stride;
  int* status;
  const DeviceTables* __restrict__ tab;
};

// y = M x for an N-vector strided through LDS, in place (M row-major [n][k]).
template <int N>
__device__ inline void lds_transform(const float* __restrict__ M, float* v, int stride) {
  float in[N];
#pragma unroll
  for (int k = 0; k < N; ++k) in[k] = v[k * stride];
  for (int n = 0; n < N; ++n) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) acc = fmaf(M[n * N + k], in[k], acc);
    v[n * stride] = acc;
  }
}

// AuxIDCT2x2(block, S) of I.2.4.2 on an 8x8 register block.
template <int S>
__device__ inline void aux_idct2x2(float (&v)[64]) {
  constexpr int h = S / 2;
  float r[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) r[i] = v[i];
#pragma unroll
  for (int y = 0; y < h; ++y)
#pragma unroll
    for (int x = 0; x < h; ++x) {
      const float c00 = v[y * 8 + x], c01 = v[y * 8 + h + x];
      const float c10 = v[(h + y) * 8 + x], c11 = v[(h + y) * 8 + h + x];
      r[(2 * y) * 8 + 2 * x] = c00 + c01 + c10 + c11;
      r[(2 * y) * 8 + 2 * x + 1] = c00 + c01 - c10 - c11;
      r[(2 * y + 1) * 8 + 2 * x] = c00 - c01 + c10 - c11;
      r[(2 * y + 1) * 8 + 2 * x + 1] = c00 - c01 - c10 + c11;
    }
#pragma unroll
  for (int i = 0; i < 64; ++i) v[i] = r[i];
}

// I.2.4.4 Identity on an 8x8 register block.
__device__ inline void identity_inverse(float (&v)[64]) {
  float k[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) k[i] = v[i];
  aux_idct2x2<2>(v);  // v's 2x2 corner now holds the four quarter DCs
  // the quarters' outputs overwrite that corner, so keep the DCs apart
  const float dcs[4] = {v[0], v[1], v[8], v[9]};
#pragma unroll
  for (int sy = 0; sy < 2; ++sy)
#pragma unroll
    for (int sx = 0; sx < 2; ++sx) {
      const float dcv = dcs[sy * 2 + sx];
      float rs = 0.0f;
#pragma unroll
      for (int iy = 0; iy < 4; ++iy)
#pragma unroll
        for (int ix = 0; ix < 4; ++ix)
          if (ix || iy) rs += k[(sy + 2 * iy) * 8 + sx + 2 * ix];
      const float s11 = dcv - rs / 16.0f;
      float o[16];
#pragma unroll
      for (int iy = 0; iy < 4; ++iy)
#pragma unroll
        for (int ix = 0; ix < 4; ++ix) o[iy * 4 + ix] = k[(sy + 2 * iy) * 8 + sx + 2 * ix] + s11;
      o[1 * 4 + 1] = s11;
      o[0] = k[(sy + 2) * 8 + sx + 2] + s11;
#pragma unroll
      for (int iy = 0; iy < 4; ++iy)
#pragma unroll
        for (int ix = 0; ix < 4; ++ix) v[(4 * sy + iy) * 8 + 4 * sx + ix] = o[iy * 4 + ix];
    }
}

__global__ __launch_bounds__(kThreads) void recon_kernel(ReconArgs a) {
  __shared__ float coef[3][32][33];
  __shared__ float s_dc[3][16];
  __shared__ float s_acmul[16];
  __shared__ uint8_t s_raw[16], s_owner[16], s_strat[16];
  __shared__ int s_ok;

  const int tid = threadIdx.x;
  const int gbx0 = 4 * blockIdx.x, gby0 = 4 * blockIdx.y;
  const int nbx = min(4, a.Wb - gbx0), nby = min(4, a.Hb - gby0);
  const int gx0 = 8 * gbx0, gy0 = 8 * gby0;
  const DeviceTables* __restrict__ T = a.tab;

  if (tid < 16) {
    const int bx = tid & 3, by = tid >> 2;
    const bool in = bx < nbx && by < nby;
    const size_t m = size_t(gby0 + by) * a.map_stride + gbx0 + bx;
    s_raw[tid] = in ? a.strategy[m] : kAbsent;
    // C.5.5: AcMul = 2^16 / (global_scale * (1 + dv)); the product is an
    // integer below 2^24, so one rounding.
    s_acmul[tid] = in ? 65536.0f / (a.gscale * float(1 + a.qf[m])) : 0.0f;
    for (int c = 0; c < 3; ++c)
      s_dc[c][tid] =
          in ? a.dc_mul[c] * float(a.dc[c][size_t(gby0 + by) * a.dc_stride + gbx0 + bx]) : 0.0f;
  }
  __syncthreads();
  if (tid == 0) s_ok = scan_region(s_raw, nbx, nby, s_owner, s_strat);
  if (tid < 16) {  // Annex G on the DC samples, with the DC factors
    const float y = s_dc[1][tid];
    s_dc[0][tid] = fmaf(a.kx_dc, y, s_dc[0][tid]);
    s_dc[2][tid] = fmaf(a.kb_dc, y, s_dc[2][tid]);
  }
  __syncthreads();
  if (!s_ok) {
    if (tid == 0) atomicOr(a.status, 1);
    for (int p = tid; p < 1024; p += kThreads) {
      const int gx = gx0 + (p & 31), gy = gy0 + (p >> 5);
      if (gx < a.W && gy < a.H)
        for (int c = 0; c < 3; ++c) a.xyb[(size_t(c) * a.H + gy) * a.xyb_stride + gx] = 0.0f;
    }
    return;
  }

  // The region's 64x64 chroma-from-luma tile.
  const size_t tile = size_t(gy0 / 64) * a.cfl_stride + gx0 / 64;
  const float kx = a.cfl_kx[tile], kb = a.cfl_kb[tile];

  // Dequantization (F.3), LLF from DC (I.2.7), chroma from luma (Annex G).
  for (int j = 0; j < 4; ++j) {
    const int p = tid + kThreads * j;
    const int py = p >> 5, px = p & 31;
    const int lb = (py >> 3) * 4 + (px >> 3);
    const int s = s_strat[lb];
    if (s == kAbsent) continue;
    const int o = s_owner[lb];
    const int x = px - 8 * (o & 3), y = py - 8 * (o >> 2);
    const int cxb = vb_bx(s), cyb = vb_by(s);
    float K[3];
    if (x < cxb && y < cyb) {
      const float* ax = cxb == 2 ? T->a16 : T->a32;
      const float* ay = cyb == 2 ? T->a16 : T->a32;
      for (int c = 0; c < 3; ++c) {
        float acc = 0.0f;
        for (int jy = 0; jy < cyb; ++jy) {
          const float fy = cyb == 1 ? 1.0f : ay[y * cyb + jy];
          for (int ix = 0; ix < cxb; ++ix) {
            const float fx = cxb == 1 ? 1.0f : ax[x * cxb + ix];
            acc = fmaf(fy * fx, s_dc[c][o + 4 * jy + ix], acc);
          }
        }
        K[c] = acc;
      }
    } else {
      const size_t g = size_t(gy0 + py) * a.ac_stride + gx0 + px;
      const int sz = 64 * cxb * cyb;
      const float* dq = T->dq + dq_off(s) + y * 8 * cxb + x;
      const float acm = s_acmul[o];
      for (int c = 0; c < 3; ++c) {
        const int q = a.ac[c][g];
        const float fq = float(q);
        const float b = (q >= -1 && q <= 1) ? fq * a.one_bias[c] : fq - 0.145f / fq;
        K[c] = b * acm * dq[c * sz];
      }
      K[0] = fmaf(kx, K[1], K[0]);
      K[2] = fmaf(kb, K[1], K[2]);
    }
    for (int c = 0; c < 3; ++c) coef[c][py][px] = K[c];
  }
  __syncthreads();

  // 8x8 transforms that are not separable matrix products: DCT2 and Identity
  // entirely, and the 2x2 corner step of DCT4 (I.2.4.2-I.2.4.4).
  if (tid < 48) {
    const int lb = tid & 15, c = tid >> 4;
    const int s = s_strat[lb];
    if ((s == 1 || s == 2 || s == 3) && s_owner[lb] == lb) {
      float* base = &coef[c][8 * (lb >> 2)][8 * (lb & 3)];
      float v[64];
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) v[r * 8 + q] = base[r * 33 + q];
      if (s == 2) {
        aux_idct2x2<2>(v);
        aux_idct2x2<4>(v);
        aux_idct2x2<8>(v);
      } else if (s == 1) {
        identity_inverse(v);
      } else {
        aux_idct2x2<2>(v);
      }
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) base[r * 33 + q] = v[r * 8 + q];
    }
  }
  __syncthreads();

  // Column pass: every column segment of every varblock (S = T_by K T_bx^T).
  for (int it = tid; it < 384; it += kThreads) {
    const int c = it >> 7, X = it & 31, br = (it >> 5) & 3;
    const int lb = br * 4 + (X >> 3);
    const int s = s_strat[lb];
    if (s == kAbsent || s == 1 || s == 2 || (s_owner[lb] >> 2) != br) continue;
    float* v = &coef[c][8 * br][X];
    const int by = vb_by(s);
    if (s == 3) lds_transform<8>(T->m4, v, 33);
    else if (by == 1) lds_transform<8>(T->t8, v, 33);
    else if (by == 2) lds_transform<16>(T->t16, v, 33);
    else lds_transform<32>(T->t32, v, 33);
  }
  __syncthreads();

  // Row pass.
  for (int it = tid; it < 384; it += kThreads) {
    const int c = it >> 7, Y = it & 31, bc = (it >> 5) & 3;
    const int lb = (Y >> 3) * 4 + bc;
    const int s = s_strat[lb];
    if (s == kAbsent || s == 1 || s == 2 || (s_owner[lb] & 3) != bc) continue;
    float* v = &coef[c][Y][8 * bc];
    const int bx = vb_bx(s);
    if (s == 3) lds_transform<8>(T->m4, v, 1);
    else if (bx == 1) lds_transform<8>(T->t8, v, 1);
    else if (bx == 2) lds_transform<16>(T->t16, v, 1);
    else lds_transform<32>(T->t32, v, 1);
  }
  __syncthreads();

  // Crop (6.2) and store.
  for (int j = 0; j < 4; ++j) {
    const int p = tid + kThreads * j;
    const int py = p >> 5, px = p & 31;
    const int gx = gx0 + px, gy = gy0 + py;
    if (gx < a.W && gy < a.H)
      for (int c = 0; c < 3; ++c) a.xyb[(size_t(c) * a.H + gy) * a.xyb_stride + gx] = coef[c][py][px];
  }
}

// ---------------------------------------------------------------------------
// Edge-preserving filter (J.2), one pass.
//
// One workgroup per 64x32 output tile (two 32x32 regions side by side); each
// thread filters an 8-pixel vertical strip of one column.  The tile and its
// filter halo are staged in LDS once:
//   s_in  input samples of columns x0-3..x0+68 and rows y0-3..y0+34 (the
//         7x8 window of every output pixel);
//   s_p   per channel, 32-bit words packing the guide bytes of 4 consecutive
//         columns, for start columns x0-4..x0+66 and rows y0-4..y0+35.
// A J.2.3 patch is 4 columns by 3 rows, so one v_sad_u8 on two such words is
// one channel's distance over one patch row.  For a window offset (cx, cy)
// the distance of the strip's pixel in row y is rs(y-1) + rs(y) + rs(y+1),
// rs(y') = sum_c sad(P_c(x-1, y'), P_c(x-1+cx, y'+cy)); the strip's ten row
// sums serve its eight overlapping patches.

struct EpfArgs {
  int W, H, Wb, Hb;
  const uint8_t* strategy;
  const uint8_t* qf;
  const uint8_t* sharp;
  size_t map_stride;
  const float* in;
  float* out;
  size_t stride;
  float minv[3], scale[3];
  uint32_t thr;  // weights below epf_weight_min: bit patterns below thr (a multiple of 2^16)
  float sharp_lut[8];
  float range_max, range_mul, quant_mul;
  float sigma_max;
  float gscale_q;  // global_scale / 65536: quant = gscale_q * (1 + dv), exact
  const int32_t* __restrict__ mul_table;
  uint8_t* guide_dbg;
  int32_t* sigma_dbg;
  int* status;
};

constexpr int kEpfTW = 64, kEpfTH = 32;  // output tile
constexpr int kInW = 72, kInH = 38;      // s_in: columns x0-3.., rows y0-3..
constexpr int kPW = 72, kPH = 40;        // s_p: start columns x0-4.., rows y0-4..
constexpr int kGW = 19;                  // packed guide words per row: columns x0-4..x0+71

__device__ inline uint32_t guide_byte(float v, float minv, float scale) {
  // J.2.2 in binary32: floor(clamp((v - min) * scale, 0, 255))
  const float sc = (v - minv) * scale;
  const float g = fminf(fmaxf(sc, 0.0f), 255.0f);
  return uint32_t(floorf(g));
}

__global__ __launch_bounds__(kThreads, 2) void epf_kernel(EpfArgs a) {
  __shared__ float s_in[3][kInH][kInW];
  __shared__ uint32_t s_p[3][kPH][kPW];
  __shared__ uint32_t s_w[3][kPH][kGW + 1];
  __shared__ float s_rng[32];
  __shared__ int s_mul[32];
  __shared__ uint8_t s_raw[2][16], s_owner[2][16], s_strat[2][16];
  __shared__ int s_ok[2];

  const int tid = threadIdx.x;
  const int x0 = kEpfTW * blockIdx.x, y0 = kEpfTH * blockIdx.y;
  const int gbx0 = x0 / 8, gby0 = y0 / 8;
  const size_t plane = size_t(a.H) * a.stride;

  // A: input samples and packed guide words (4 columns per word).
  for (int it = tid; it < kPH * kGW; it += kThreads) {
    const int v = it / kGW, g = it % kGW;
    const int gy = mirror(y0 - 4 + v, a.H);
    uint32_t w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int lxx = x0 - 4 + 4 * g + j;
      const int gx = mirror(lxx, a.W);
      const float* p = a.in + size_t(gy) * a.stride + gx;
      const float v0 = p[0], v1 = p[plane], v2 = p[2 * plane];
      w0 |= guide_byte(v0, a.minv[0], a.scale[0]) << (8 * j);
      w1 |= guide_byte(v1, a.minv[1], a.scale[1]) << (8 * j);
      w2 |= guide_byte(v2, a.minv[2], a.scale[2]) << (8 * j);
      const int ci = 4 * g + j - 1, ri = v - 1;
      if (ci >= 0 && ci < kInW && ri >= 0 && ri < kInH) {
        s_in[0][ri][ci] = v0;
        s_in[1][ri][ci] = v1;
        s_in[2][ri][ci] = v2;
      }
    }
    s_w[0][v][g] = w0;
    s_w[1][v][g] = w1;
    s_w[2][v][g] = w2;
  }
  if (tid < 32) {
    const int r = tid >> 4, lb = tid & 15;
    const int bx = gbx0 + 4 * r + (lb & 3), by = gby0 + (lb >> 2);
    s_raw[r][lb] = (bx < a.Wb && by < a.Hb) ? a.strategy[size_t(by) * a.map_stride + bx] : kAbsent;
  }
  __syncthreads();

  // B: guide words at every start column; C: region scans.
  for (int it = tid; it < 3 * kPH * (kPW - 1); it += kThreads) {
    const int c = it / (kPH * (kPW - 1));
    const int rem = it % (kPH * (kPW - 1));
    const int v = rem / (kPW - 1), u = rem % (kPW - 1);
    s_p[c][v][u] = __builtin_amdgcn_alignbyte(s_w[c][v][(u >> 2) + 1], s_w[c][v][u >> 2], u & 3);
  }
  if ((tid & 63) == 0 && tid < 128) {
    const int r = tid >> 6;
    // a region right of the frame has no blocks: the scan marks all absent
    const int nbx = max(0, min(4, a.Wb - (gbx0 + 4 * r))), nby = min(4, a.Hb - gby0);
    s_ok[r] = scan_region(s_raw[r], nbx, nby, s_owner[r], s_strat[r]);
  }
  // Per-block range of `scaled` (J.2.4) over the block's pixels inside the
  // frame: eight lanes per block, one row each, reduced across the lanes.
  {
    const int b = tid >> 3, r = tid & 7;
    const int bxl = b & 7, byl = b >> 3;
    const int gy = y0 + 8 * byl + r;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (gy < a.H)
      for (int j = 0; j < 8; ++j) {
        if (x0 + 8 * bxl + j >= a.W) break;
        for (int c = 0; c < 3; ++c) {
          const float sc = (s_in[c][3 + 8 * byl + r][3 + 8 * bxl + j] - a.minv[c]) * a.scale[c];
          lo[c] = fminf(lo[c], sc);
          hi[c] = fmaxf(hi[c], sc);
        }
      }
    float rg = 0.0f;
    for (int c = 0; c < 3; ++c) {
      for (int m = 1; m < 8; m <<= 1) {
        lo[c] = fminf(lo[c], __shfl_xor(lo[c], m, 8));
        hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], m, 8));
      }
      if (hi[c] >= lo[c]) rg = fmaxf(rg, hi[c] - lo[c]);
    }
    if (r == 0) s_rng[b] = rg;
  }
  __syncthreads();

  // D: sigma and mul per block; mul * 64 is stored, 1 marks "not filtered".
  if (tid < 32) {
    const int bxl = tid & 7, byl = tid >> 3;
    const int r = bxl >> 2, lb = byl * 4 + (bxl & 3);
    const int bx = gbx0 + bxl, by = gby0 + byl;
    int sig = 0;
    if (!s_ok[r] && lb == 0) atomicOr(a.status, 1);
    if (s_ok[r] && s_strat[r][lb] != kAbsent) {
      float rg = 0.0f;
      for (int m = 0; m < 16; ++m)
        if (s_owner[r][m] == s_owner[r][lb]) rg = fmaxf(rg, s_rng[(m >> 2) * 8 + 4 * r + (m & 3)]);
      const size_t mi = size_t(by) * a.map_stride + bx;
      float sg = fminf(rg, a.range_max) * a.range_mul * a.sharp_lut[a.sharp[mi] & 7];
      sg = fminf(sg, a.gscale_q * float(1 + a.qf[mi]) * a.quant_mul);
      sg = fminf(sg, a.sigma_max);
      sig = int(sg);  // truncation; sg >= 0
    }
    s_mul[tid] = sig >= 16 ? a.mul_table[sig] * 64 : 1;
    if (a.sigma_dbg && bx < a.Wb && by < a.Hb) a.sigma_dbg[size_t(by) * a.Wb + bx] = sig;
  }
  __syncthreads();

  // E: the strip of 8 pixels of column x.
  const int lx = tid & 63, strip = tid >> 6;
  const int x = x0 + lx, ys = y0 + 8 * strip;
  if (x >= a.W || ys >= a.H) return;
  const int nrows = min(8, a.H - ys);
  const int mul64 = s_mul[strip * 8 + (lx >> 3)];
  float* o0 = a.out + size_t(ys) * a.stride + x;
  if (a.guide_dbg) {
    const int wg = (lx + 4) >> 2, sh = 8 * ((lx + 4) & 3);
    for (int i = 0; i < nrows; ++i)
      for (int c = 0; c < 3; ++c)
        a.guide_dbg[(size_t(c) * a.H + ys + i) * a.W + x] =
            uint8_t(s_w[c][8 * strip + 4 + i][wg] >> sh);
  }
  if (mul64 > 0) {  // sigma < 16: the pass leaves the pixel unchanged
    for (int i = 0; i < nrows; ++i)
      for (int c = 0; c < 3; ++c)
        o0[c * plane + size_t(i) * a.stride] = s_in[c][8 * strip + 3 + i][lx + 3];
    return;
  }
  // Weight(sad, mul) of J.2.4: ((min(sad,507) << 6) * mul >> 16) + (127 << 7),
  // placed in the top half of a binary32 pattern, equals
  // (min(sad,507) * 64 mul + (127 << 23)) with the low 16 bits cleared.
  constexpr int kC = 127 << 23;
  const uint32_t thr = a.thr;
  uint32_t ref[10][3];
#pragma unroll
  for (int j = 0; j < 10; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) ref[j][c] = s_p[c][8 * strip + 3 + j][lx + 3];
  float acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[i][c] = 0.0f;

  for (int cx = -3; cx <= 4; ++cx) {
    uint32_t nb[16][3];
    float inp[14][3];
#pragma unroll
    for (int j = 0; j < 16; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) nb[j][c] = s_p[c][8 * strip + j][lx + 3 + cx];
#pragma unroll
    for (int j = 0; j < 14; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) inp[j][c] = s_in[c][8 * strip + j][lx + 3 + cx];
#pragma unroll
    for (int cy = -3; cy <= 3; ++cy) {
      uint32_t rs[10];
#pragma unroll
      for (int j = 0; j < 10; ++j) {
        uint32_t s = __builtin_amdgcn_sad_u8(ref[j][0], nb[j + cy + 3][0], 0u);
        s = __builtin_amdgcn_sad_u8(ref[j][1], nb[j + cy + 3][1], s);
        rs[j] = __builtin_amdgcn_sad_u8(ref[j][2], nb[j + cy + 3][2], s);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint32_t sad = min(rs[i] + rs[i + 1] + rs[i + 2], 507u);
        const uint32_t t = uint32_t(__mul24(int(sad), mul64) + kC);
        const float w = __uint_as_float(t >= thr ? (t & 0xFFFF0000u) : 0u);
        acc[i][3] += w;
        acc[i][0] = fmaf(w, inp[i + cy + 3][0], acc[i][0]);
        acc[i][1] = fmaf(w, inp[i + cy + 3][1], acc[i][1]);
        acc[i][2] = fmaf(w, inp[i + cy + 3][2], acc[i][2]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < nrows)
#pragma unroll
      for (int c = 0; c < 3; ++c) o0[c * plane + size_t(i) * a.stride] = acc[i][c] / acc[i][3];
}

// ---------------------------------------------------------------------------
// Gaborish (J.4) + XYB -> RGB (L.2) + output encoding.

struct FinishArgs {
  int W, H;
  const float* in;
  size_t stride;
  int gab;
  float k0[3], k1[3], k2[3];  // normalized centre, edge, corner weights
  float m[9];                 // inverse opsin matrix / (target_nits_div50 * 50 / 250) / 255
  float bias[3];
  int format;
  void* out[3];
  size_t out_stride;
};

__device__ inline float srgb_encode(float v) {
  v = fminf(fmaxf(v, 0.0f), 1.0f);
  return v <= 0.0031308f ? 12.92f * v : 1.055f * powf(v, 1.0f / 2.4f) - 0.055f;
}

__global__ __launch_bounds__(kThreads) void finish_kernel(FinishArgs a) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= a.W || y >= a.H) return;
  const size_t plane = size_t(a.H) * a.stride;
  float v[3];
  if (a.gab) {
    const int xm = mirror(x - 1, a.W), xp = mirror(x + 1, a.W);
    const int ym = mirror(y - 1, a.H), yp = mirror(y + 1, a.H);
    for (int c = 0; c < 3; ++c) {
      const float* p = a.in + c * plane;
      const float* rm = p + size_t(ym) * a.stride;
      const float* r0 = p + size_t(y) * a.stride;
      const float* rp = p + size_t(yp) * a.stride;
      const float edge = (rm[x] + r0[xm]) + (r0[xp] + rp[x]);
      const float corner = (rm[xm] + rm[xp]) + (rp[xm] + rp[xp]);
      v[c] = fmaf(a.k0[c], r0[x], fmaf(a.k1[c], edge, a.k2[c] * corner));
    }
  } else {
    for (int c = 0; c < 3; ++c) v[c] = a.in[c * plane + size_t(y) * a.stride + x];
  }
  const float gr = v[1] + v[0], gg = v[1] - v[0], gb = v[2];
  const float mr = fmaf(gr * gr, gr, a.bias[0]);
  const float mg = fmaf(gg * gg, gg, a.bias[1]);
  const float mb = fmaf(gb * gb, gb, a.bias[2]);
  float rgb[3];
  for (int r = 0; r < 3; ++r)
    rgb[r] = fmaf(a.m[3 * r], mr, fmaf(a.m[3 * r + 1], mg, a.m[3 * r + 2] * mb));
  const size_t o = size_t(y) * a.out_stride + x;
  if (a.format == JXLR_OUT_F32) {
    for (int c = 0; c < 3; ++c) static_cast<float*>(a.out[c])[o] = rgb[c];
  } else if (a.format == JXLR_OUT_U8_SRGB) {
    for (int c = 0; c < 3; ++c)
      static_cast<uint8_t*>(a.out[c])[o] = uint8_t(floorf(srgb_encode(rgb[c]) * 255.0f + 0.5f));
  } else {
    for (int c = 0; c < 3; ++c)
      static_cast<uint16_t*>(a.out[c])[o] =
          uint16_t(floorf(srgb_encode(rgb[c]) * 65535.0f + 0.5f));
  }
}

// ---------------------------------------------------------------------------
// Host side.

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

jxlr_status check_params(const jxlr_frame_params* p) {
  if (!p) return JXLR_E_NULL;
  if (p->xsize == 0 || p->ysize == 0 || p->xsize > JXLR_MAX_DIM || p->ysize > JXLR_MAX_DIM)
    return JXLR_E_SIZE;
  if (p->global_scale < 1 || p->global_scale > 65536) return JXLR_E_PARAM;
  for (int c = 0; c < 3; ++c)
    if (p->extra_levels[c] < 0 || p->extra_levels[c] > 3) return JXLR_E_PARAM;
  if (p->epf_iters < 0 || p->epf_iters > 3) return JXLR_E_PARAM;
  if (!(p->epf_weight_min <= 1.0f)) return JXLR_E_PARAM;
  if (p->epf_sigma_max < 0 || p->epf_sigma_max > 672) return JXLR_E_PARAM;
  if (p->epf_sigma_shift < 0 || p->epf_sigma_shift > 8) return JXLR_E_PARAM;
  if (p->target_nits_div50 < 1) return JXLR_E_PARAM;
  if (p->out_format < JXLR_OUT_F32 || p->out_format > JXLR_OUT_U16_SRGB) return JXLR_E_PARAM;
  return JXLR_OK;
}

int blocks_of(uint32_t v) { return int((v + 7) / 8); }

jxlr_status check_maps_io(const jxlr_frame_params* p, const jxlr_frame_io* io, bool need_sharp) {
  if (!io || !io->strategy || !io->qf_minus_1 || (need_sharp && !io->sharpness))
    return JXLR_E_NULL;
  if (io->map_stride < size_t(blocks_of(p->xsize))) return JXLR_E_SIZE;
  return JXLR_OK;
}

jxlr_status launch_status(hipError_t e) { return e == hipSuccess ? JXLR_OK : JXLR_E_HIP; }

}  // namespace

extern "C" {

const char* jxlr_status_string(jxlr_status s) {
  switch (s) {
    case JXLR_OK: return "ok";
    case JXLR_E_NULL: return "null pointer";
    case JXLR_E_SIZE: return "size or stride out of range";
    case JXLR_E_STRATEGY: return "transform type not supported";
    case JXLR_E_ALIGN: return "varblock misaligned, out of bounds or overlapping";
    case JXLR_E_QUANT: return "quant field not uniform within a varblock";
    case JXLR_E_DEQUANT: return "dequantization matrix entry not positive and finite";
    case JXLR_E_PARAM: return "frame parameter out of range";
    case JXLR_E_WORKSPACE: return "workspace too small";
    case JXLR_E_HIP: return "HIP runtime error";
    case JXLR_E_DEVICE_VALIDATION: return "device found an ill-formed DctSelect map";
  }
  return "unknown status";
}

jxlr_status jxlr_params_default(jxlr_frame_params* p, uint32_t xsize, uint32_t ysize) {
  if (!p) return JXLR_E_NULL;
  std::memset(p, 0, sizeof(*p));
  p->xsize = xsize;
  p->ysize = ysize;
  p->global_scale = 1;
  const float w[3] = {4096.0f, 512.0f, 256.0f};  // C.4.1, global_scale = quant_dc = 1
  for (int c = 0; c < 3; ++c) p->dc_mul[c] = w[c];
  p->kx_dc = 0.0f;                               // x_factor_dc = 128
  p->kb_dc = 0.935669f;                          // b_factor_dc = 128
  p->gab = 1;
  for (int c = 0; c < 3; ++c) {
    p->gab_w1[c] = 0.115169525f;
    p->gab_w2[c] = 0.061248592f;
  }
  p->epf_iters = 1;
  p->epf_weight_min = 0.3f;
  p->epf_scale[0] = 899.676941f;
  p->epf_scale[1] = 111.965157f;
  p->epf_scale[2] = 45.275791f;
  for (int i = 0; i < 8; ++i) p->epf_sharp_lut[i] = float(i) / 7.0f;
  p->epf_range_max = 70.0f;
  p->epf_range_mul = 12.6f;
  p->epf_quant_mul = 20.0f;
  p->epf_sigma_max = 170;
  p->epf_sigma_shift = 0;
  const float m[9] = {2542.56835937500000f, -2326.53173828125000f, 44.17734527587891f,
                      -698.04852294921875f, 1012.71777343750000f,  -76.22974395751953f,
                      -827.36480712890625f, 709.83502197265625f,   451.38488769531250f};
  std::memcpy(p->opsin_inv, m, sizeof(m));
  p->opsin_bias[0] = -0.00100549f;
  p->opsin_bias[1] = -0.00100549f;
  p->opsin_bias[2] = -0.00094081f;
  p->target_nits_div50 = 5;
  p->out_format = JXLR_OUT_F32;
  return JXLR_OK;
}

jxlr_status jxlr_create(jxlr_ctx** out, int device) {
  if (!out) return JXLR_E_NULL;
  *out = nullptr;
  DeviceGuard g(device);
  if (!g.ok) return JXLR_E_HIP;
  auto* host = new DeviceTables;
  if (!jxlr::build_tables(host)) {
    delete host;
    return JXLR_E_DEQUANT;
  }
  auto* ctx = new jxlr_ctx{device, nullptr, nullptr};
  hipError_t e = hipMalloc(&ctx->tables, sizeof(DeviceTables));
  if (e == hipSuccess) e = hipMalloc(&ctx->status, sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(ctx->tables, host, sizeof(DeviceTables), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(ctx->status, 0, sizeof(int));
  delete host;
  if (e != hipSuccess) {
    jxlr_destroy(ctx);
    return JXLR_E_HIP;
  }
  *out = ctx;
  return JXLR_OK;
}

void jxlr_destroy(jxlr_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  if (ctx->tables) (void)hipFree(ctx->tables);
  if (ctx->status) (void)hipFree(ctx->status);
  delete ctx;
}

jxlr_status jxlr_validate_maps_host(const jxlr_frame_params* p, const uint8_t* strategy,
                                    const uint8_t* qf, const uint8_t* sharp, size_t stride) {
  jxlr_status st = check_params(p);
  if (st) return st;
  if (!strategy || !qf) return JXLR_E_NULL;
  const int Wb = blocks_of(p->xsize), Hb = blocks_of(p->ysize);
  if (stride < size_t(Wb)) return JXLR_E_SIZE;
  std::vector<uint8_t> covered(size_t(Wb) * Hb, 0);
  for (int by = 0; by < Hb; ++by)
    for (int bx = 0; bx < Wb; ++bx) {
      if (sharp && sharp[size_t(by) * stride + bx] > 7) return JXLR_E_PARAM;
      if (covered[size_t(by) * Wb + bx]) continue;
      const int s = strategy[size_t(by) * stride + bx];
      if (s >= jxlr::kNumStrategies) return JXLR_E_STRATEGY;
      const int cx = vb_bx(s), cy = vb_by(s);
      if (bx % cx || by % cy || bx + cx > Wb || by + cy > Hb) return JXLR_E_ALIGN;
      const uint8_t q = qf[size_t(by) * stride + bx];
      for (int j = 0; j < cy; ++j)
        for (int i = 0; i < cx; ++i) {
          uint8_t& cv = covered[size_t(by + j) * Wb + bx + i];
          if (cv) return JXLR_E_ALIGN;
          cv = 1;
          if (qf[size_t(by + j) * stride + bx + i] != q) return JXLR_E_QUANT;
        }
    }
  return JXLR_OK;
}

size_t jxlr_workspace_bytes(const jxlr_frame_params* p) {
  if (check_params(p) != JXLR_OK) return 0;
  const size_t one = (size_t(3) * p->xsize * p->ysize * sizeof(float) + 255) & ~size_t(255);
  return p->epf_iters > 0 ? 2 * one : one;
}

jxlr_status jxlr_reconstruct(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                             float* xyb, size_t xyb_stride, hipStream_t stream) {
  if (!ctx || !xyb) return JXLR_E_NULL;
  jxlr_status st = check_params(p);
  if (st) return st;
  if ((st = check_maps_io(p, io, false))) return st;
  for (int c = 0; c < 3; ++c)
    if (!io->ac[c] || !io->dc[c]) return JXLR_E_NULL;
  if (!io->cfl_kx || !io->cfl_kb) return JXLR_E_NULL;
  const int Wb = blocks_of(p->xsize), Hb = blocks_of(p->ysize);
  if (io->ac_stride < size_t(8 * Wb) || io->dc_stride < size_t(Wb) ||
      io->cfl_stride < size_t((p->xsize + 63) / 64) || xyb_stride < p->xsize)
    return JXLR_E_SIZE;
  ReconArgs a{};
  a.W = int(p->xsize);
  a.H = int(p->ysize);
  a.Wb = Wb;
  a.Hb = Hb;
  for (int c = 0; c < 3; ++c) {
    a.ac[c] = io->ac[c];
    a.dc[c] = io->dc[c];
    a.dc_mul[c] = p->dc_mul[c] / float(1 << p->extra_levels[c]);
  }
  a.ac_stride = io->ac_stride;
  a.dc_stride = io->dc_stride;
  a.strategy = io->strategy;
  a.qf = io->qf_minus_1;
  a.map_stride = io->map_stride;
  a.cfl_kx = io->cfl_kx;
  a.cfl_kb = io->cfl_kb;
  a.cfl_stride = io->cfl_stride;
  a.kx_dc = p->kx_dc;
  a.kb_dc = p->kb_dc;
  a.gscale = float(p->global_scale);
  const double kOneBias[3] = {0.05465007330715401, 0.07005449891748593, 0.049935103337343655};
  for (int c = 0; c < 3; ++c) a.one_bias[c] = float(1.0 - kOneBias[c]);
  a.xyb = xyb;
  a.xyb_stride = xyb_stride;
  a.status = ctx->status;
  a.tab = ctx->tables;
  DeviceGuard g(ctx->device);
  if (!g.ok) return JXLR_E_HIP;
  dim3 grid((Wb + 3) / 4, (Hb + 3) / 4);
  hipLaunchKernelGGL(recon_kernel, grid, dim3(kThreads), 0, stream, a);
  return launch_status(hipGetLastError());
}

jxlr_status jxlr_epf_pass(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                          const float* in, float* out, size_t stride, uint8_t* guide_dbg,
                          int32_t* sigma_dbg, hipStream_t stream) {
  if (!ctx || !in || !out) return JXLR_E_NULL;
  jxlr_status st = check_params(p);
  if (st) return st;
  if ((st = check_maps_io(p, io, true))) return st;
  if (stride < p->xsize) return JXLR_E_SIZE;
  EpfArgs a{};
  a.W = int(p->xsize);
  a.H = int(p->ysize);
  a.Wb = blocks_of(p->xsize);
  a.Hb = blocks_of(p->ysize);
  a.strategy = io->strategy;
  a.qf = io->qf_minus_1;
  a.sharp = io->sharpness;
  a.map_stride = io->map_stride;
  a.in = in;
  a.out = out;
  a.stride = stride;
  // J.2.1: intensity_multiplier3 = cbrt(target_nits_div50 * 50 / 250)
  const double im3 = std::cbrt(p->target_nits_div50 * 50.0 / 250.0);
  a.minv[0] = float(-0.03 * im3);
  a.minv[1] = a.minv[2] = 0.0f;
  for (int c = 0; c < 3; ++c) a.scale[c] = p->epf_scale[c];
  {
    // weights w < epf_weight_min are dropped; the weights are multiples of
    // 2^16 in bit pattern, so compare against the next such multiple
    float wm = p->epf_weight_min;
    uint32_t bits;
    std::memcpy(&bits, &wm, 4);
    a.thr = wm <= 0.0f ? 0u : ((bits + 0xFFFFu) & 0xFFFF0000u);
  }
  for (int i = 0; i < 8; ++i) a.sharp_lut[i] = p->epf_sharp_lut[i];
  a.range_max = p->epf_range_max;
  a.range_mul = p->epf_range_mul;
  a.quant_mul = p->epf_quant_mul;
  a.sigma_max = float(p->epf_sigma_max);
  a.gscale_q = float(p->global_scale) / 65536.0f;
  a.mul_table = ctx->tables->mul_table[p->epf_sigma_shift];
  a.guide_dbg = guide_dbg;
  a.sigma_dbg = sigma_dbg;
  a.status = ctx->status;
  DeviceGuard g(ctx->device);
  if (!g.ok) return JXLR_E_HIP;
  dim3 grid((p->xsize + kEpfTW - 1) / kEpfTW, (p->ysize + kEpfTH - 1) / kEpfTH);
  hipLaunchKernelGGL(epf_kernel, grid, dim3(kThreads), 0, stream, a);
  return launch_status(hipGetLastError());
}

jxlr_status jxlr_finish(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                        const float* xyb, size_t stride, hipStream_t stream) {
  if (!ctx || !xyb || !io) return JXLR_E_NULL;
  jxlr_status st = check_params(p);
  if (st) return st;
  for (int c = 0; c < 3; ++c)
    if (!io->out[c]) return JXLR_E_NULL;
  if (stride < p->xsize || io->out_stride < p->xsize) return JXLR_E_SIZE;
  FinishArgs a{};
  a.W = int(p->xsize);
  a.H = int(p->ysize);
  a.in = xyb;
  a.stride = stride;
  a.gab = p->gab;
  for (int c = 0; c < 3; ++c) {
    // J.4: weights 1, w1, w2 rescaled to sum to 1
    const double w1 = p->gab_w1[c], w2 = p->gab_w2[c];
    const double norm = 1.0 + 4.0 * w1 + 4.0 * w2;
    a.k0[c] = float(1.0 / norm);
    a.k1[c] = float(w1 / norm);
    a.k2[c] = float(w2 / norm);
    a.bias[c] = p->opsin_bias[c];
  }
  // L.2: divide by target_nits_div50 * 50 / 250, then by 255 for [0, 1]
  const double div = p->target_nits_div50 * 50.0 / 250.0 * 255.0;
  for (int i = 0; i < 9; ++i) a.m[i] = float(double(p->opsin_inv[i]) / div);
  a.format = p->out_format;
  for (int c = 0; c < 3; ++c) a.out[c] = io->out[c];
  a.out_stride = io->out_stride;
  DeviceGuard g(ctx->device);
  if (!g.ok) return JXLR_E_HIP;
  dim3 grid((p->xsize + 63) / 64, (p->ysize + 3) / 4);
  hipLaunchKernelGGL(finish_kernel, grid, dim3(kThreads), 0, stream, a);
  return launch_status(hipGetLastError());
}

jxlr_status jxlr_decode(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                        void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx || !io || !ws) return JXLR_E_NULL;
  jxlr_status st = check_params(p);
  if (st) return st;
  const size_t need = jxlr_workspace_bytes(p);
  if (ws_bytes < need) return JXLR_E_WORKSPACE;
  float* bufa = static_cast<float*>(ws);
  float* bufb = reinterpret_cast<float*>(static_cast<char*>(ws) + need / 2);
  const size_t stride = p->xsize;
  if ((st = jxlr_reconstruct(ctx, p, io, bufa, stride, stream))) return st;
  for (int it = 0; it < p->epf_iters; ++it) {
    if ((st = jxlr_epf_pass(ctx, p, io, bufa, bufb, stride, nullptr, nullptr, stream))) return st;
    std::swap(bufa, bufb);
  }
  return jxlr_finish(ctx, p, io, bufa, stride, stream);
}

jxlr_status jxlr_get_device_status(jxlr_ctx* ctx, hipStream_t stream) {
  if (!ctx) return JXLR_E_NULL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return JXLR_E_HIP;
  int h = 0;
  if (hipMemcpyAsync(&h, ctx->status, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return JXLR_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return JXLR_E_HIP;
  if (h) {
    if (hipMemsetAsync(ctx->status, 0, sizeof(int), stream) != hipSuccess) return JXLR_E_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return JXLR_E_HIP;
    return JXLR_E_DEVICE_VALIDATION;
  }
  return JXLR_OK;
}

}  // extern "C"
