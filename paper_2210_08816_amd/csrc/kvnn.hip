// The steady-state predictor of kvnn.h: a three-level 3-D U-Net trained by
// hand-written forward and backward kernels.  The 3x3x3 convolutions and
// their input and weight gradients are implicit GEMMs on the FP32 matrix
// cores (v_mfma_f32_16x16x4) over LDS-staged voxel tiles; the 1x1x1 head is
// direct.  Their weights are the BF16-rounded master weights, products are
// accumulated in FP32.  Reductions (weight and bias gradients, the loss) are
// computed in a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/kvnn.h"

namespace {

constexpr int NT = 256;  // threads per block of every kernel here

__device__ __forceinline__ float bf16_round(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b & 0x7f800000u) == 0x7f800000u) return x;  // inf and nan unchanged
  b = (b + 0x7fffu + ((b >> 16) & 1u)) & 0xffff0000u;
  return __uint_as_float(b);
}

// ---- convolutions ----------------------------------------------------------------
// out[b][co][v] = act(bias[co] + sum_ci sum_t w[co][ci][t] in[b][ci][v + t - H])
// grid (ceil(V/NT), co_n/COB, batch); each lane computes COB channels of one voxel.
template <int KS, bool RELU, int COB>
__global__ void __launch_bounds__(NT) conv_fwd(const float* __restrict__ in, int ci_n, const float* __restrict__ w,
                                               const float* __restrict__ bias, float* __restrict__ out, int co_n,
                                               int R) {
  constexpr int T = KS * KS * KS, H = KS / 2;
  const int V = R * R * R;
  const int v = blockIdx.x * NT + threadIdx.x;
  const int co0 = blockIdx.y * COB, b = blockIdx.z;
  if (v >= V) return;
  const int x = v % R, y = (v / R) % R, z = v / (R * R);
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = bias[co0 + c];
  const float* src = in + (size_t)b * ci_n * V;
  for (int ci = 0; ci < ci_n; ++ci, src += V) {
    const float* wk = w + ((size_t)co0 * ci_n + ci) * T;
#pragma unroll
    for (int dz = 0; dz < KS; ++dz) {
      const int zz = z + dz - H;
      if (zz < 0 || zz >= R) continue;
#pragma unroll
      for (int dy = 0; dy < KS; ++dy) {
        const int yy = y + dy - H;
        if (yy < 0 || yy >= R) continue;
#pragma unroll
        for (int dx = 0; dx < KS; ++dx) {
          const int xx = x + dx - H;
          if (xx < 0 || xx >= R) continue;
          const float s = src[(zz * R + yy) * R + xx];
          const int t = (dz * KS + dy) * KS + dx;
#pragma unroll
          for (int c = 0; c < COB; ++c) acc[c] += wk[(size_t)c * ci_n * T + t] * s;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < COB; ++c) {
    float a = acc[c];
    if (RELU) a = a > 0.f ? a : 0.f;
    out[((size_t)b * co_n + co0 + c) * V + v] = a;
  }
}

// din[b][ci][v] = sum_co sum_t w[co][ci][t] dout[b][co][v - t + H]
// grid (ceil(V/NT), ci_n/CIB, batch)
template <int KS, int CIB>
__global__ void __launch_bounds__(NT) conv_bwd_data(const float* __restrict__ dout, int co_n,
                                                    const float* __restrict__ w, float* __restrict__ din, int ci_n,
                                                    int R) {
  constexpr int T = KS * KS * KS, H = KS / 2;
  const int V = R * R * R;
  const int v = blockIdx.x * NT + threadIdx.x;
  const int ci0 = blockIdx.y * CIB, b = blockIdx.z;
  if (v >= V) return;
  const int x = v % R, y = (v / R) % R, z = v / (R * R);
  float acc[CIB];
#pragma unroll
  for (int c = 0; c < CIB; ++c) acc[c] = 0.f;
  const float* src = dout + (size_t)b * co_n * V;
  for (int co = 0; co < co_n; ++co, src += V) {
    const float* wk = w + ((size_t)co * ci_n + ci0) * T;
#pragma unroll
    for (int dz = 0; dz < KS; ++dz) {
      const int zz = z - dz + H;
      if (zz < 0 || zz >= R) continue;
#pragma unroll
      for (int dy = 0; dy < KS; ++dy) {
        const int yy = y - dy + H;
        if (yy < 0 || yy >= R) continue;
#pragma unroll
        for (int dx = 0; dx < KS; ++dx) {
          const int xx = x - dx + H;
          if (xx < 0 || xx >= R) continue;
          const float s = src[(zz * R + yy) * R + xx];
          const int t = (dz * KS + dy) * KS + dx;
#pragma unroll
          for (int c = 0; c < CIB; ++c) acc[c] += wk[c * T + t] * s;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CIB; ++c) din[((size_t)b * ci_n + ci0 + c) * V + v] = acc[c];
}

// Weight-gradient partial sums over one slice of the (batch, voxel) range:
// part[s][co][ci][t] = sum_{(b,v) in slice s} dout[b][co][v] in[b][ci][v + t - H]
// grid (ci_n, co_n/COB, S).  The block sums its lanes in a fixed order.
template <int KS, int COB>
__global__ void __launch_bounds__(NT) conv_bwd_weight(const float* __restrict__ in, int ci_n,
                                                      const float* __restrict__ dout, int co_n, int batch, int R,
                                                      float* __restrict__ part, float* __restrict__ bpart) {
  constexpr int T = KS * KS * KS, H = KS / 2;
  __shared__ float red[NT / 64][COB * (T + 1)];
  const int ci = blockIdx.x, co0 = blockIdx.y * COB, s = blockIdx.z, S = gridDim.z;
  const int V = R * R * R;
  const int total = batch * V;
  const int chunk = (total + S - 1) / S;
  const int e0 = s * chunk, e1 = min(total, e0 + chunk);
  float acc[COB][T], accb[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) {
    accb[c] = 0.f;
#pragma unroll
    for (int t = 0; t < T; ++t) acc[c][t] = 0.f;
  }
  for (int e = e0 + (int)threadIdx.x; e < e1; e += NT) {
    const int b = e / V, v = e - b * V;
    const int x = v % R, y = (v / R) % R, z = v / (R * R);
    float g[COB];
#pragma unroll
    for (int c = 0; c < COB; ++c) {
      g[c] = dout[((size_t)b * co_n + co0 + c) * V + v];
      accb[c] += g[c];
    }
    const float* src = in + ((size_t)b * ci_n + ci) * V;
#pragma unroll
    for (int dz = 0; dz < KS; ++dz) {
      const int zz = z + dz - H;
      const bool zin = zz >= 0 && zz < R;
#pragma unroll
      for (int dy = 0; dy < KS; ++dy) {
        const int yy = y + dy - H;
        const bool yin = zin && yy >= 0 && yy < R;
#pragma unroll
        for (int dx = 0; dx < KS; ++dx) {
          const int xx = x + dx - H;
          const float sv = (yin && xx >= 0 && xx < R) ? src[(zz * R + yy) * R + xx] : 0.f;
          const int t = (dz * KS + dy) * KS + dx;
#pragma unroll
          for (int c = 0; c < COB; ++c) acc[c][t] += g[c] * sv;
        }
      }
    }
  }
  // wave sums (butterfly), then the waves in order; column T is the bias
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < COB; ++c)
#pragma unroll
    for (int t = 0; t <= T; ++t) {
      float a = t < T ? acc[c][t] : accb[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      if (lane == 0) red[wv][c * (T + 1) + t] = a;
    }
  __syncthreads();
  for (int q = threadIdx.x; q < COB * (T + 1); q += NT) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) a += red[k][q];
    const int c = q / (T + 1), t = q - c * (T + 1);
    if (t < T) part[(((size_t)s * co_n + co0 + c) * ci_n + ci) * T + t] = a;
    else if (ci == 0) bpart[(size_t)s * co_n + co0 + c] = a;
  }
}

// ---- voxel tiles of the 3x3x3 convolutions ---------------------------------------------
// A block owns an 8 x 8 x 4 voxel tile.  Input channels are staged CCH at a
// time as (8+2) x (8+2) x (4+2) halo tiles in LDS (zero outside the domain);
// the next channels' values are loaded into registers while the current ones
// are consumed, so every tap is an LDS read at a constant offset.
constexpr int TX = 8, TY = 8, TZ = 4, HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HALO = HX * HY * HZ;
constexpr int CCH = 4;                                   // input channels per LDS stage
constexpr int PF = (CCH * HALO + NT - 1) / NT;           // staged values per lane

struct TileIdx {
  int x0, y0, z0, tx, ty, tz;
};
__device__ __forceinline__ TileIdx tile_of(int t, int R) {
  const int nt = (R + TX - 1) / TX, ny = (R + TY - 1) / TY;
  TileIdx q;
  q.x0 = (t % nt) * TX;
  q.y0 = ((t / nt) % ny) * TY;
  q.z0 = (t / (nt * ny)) * TZ;
  q.tx = threadIdx.x % TX;
  q.ty = (threadIdx.x / TX) % TY;
  q.tz = threadIdx.x / (TX * TY);
  return q;
}
__device__ __forceinline__ int tiles_of(int R) {
  return ((R + TX - 1) / TX) * ((R + TY - 1) / TY) * ((R + TZ - 1) / TZ);
}

// Values of channels c0 .. c0+CCH-1 on the halo of tile q (zero outside the
// domain or past the last channel) into registers, then into LDS.
__device__ __forceinline__ void halo_load(const float* __restrict__ src, int c0, int c_n, int R, const TileIdx& q,
                                          float (&r)[PF]) {
  const int V = R * R * R;
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int e = threadIdx.x + k * NT;
    float v = 0.f;
    if (e < CCH * HALO) {
      const int cc = e / HALO, h = e - cc * HALO;
      const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
      const int gx = q.x0 + hx - 1, gy = q.y0 + hy - 1, gz = q.z0 + hz - 1;
      if (c0 + cc < c_n && gx >= 0 && gx < R && gy >= 0 && gy < R && gz >= 0 && gz < R)
        v = src[(size_t)(c0 + cc) * V + (gz * R + gy) * R + gx];
    }
    r[k] = v;
  }
}
__device__ __forceinline__ void halo_store(float* __restrict__ buf, const float (&r)[PF]) {
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int e = threadIdx.x + k * NT;
    if (e < CCH * HALO) buf[e] = r[k];
  }
}

// ---- 3x3x3 convolutions as implicit GEMMs on the FP32 matrix cores ----------------
// v_mfma_f32_16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[4 (l / 16) + e][l % 16], e = 0..3.
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int MO = 16;          // output channels per block (one MFMA row block)
constexpr int KST = CCH * 27;   // GEMM k per LDS stage: CCH channels x 27 taps
constexpr int PW = (KST * MO + NT - 1) / NT;

__device__ __forceinline__ int tap_offset(int t) { return ((t / 9) * HY + (t / 3) % 3) * HX + t % 3; }
__device__ __forceinline__ int voxel_offset(int nn) { return ((nn >> 6) * HY + ((nn >> 3) & 7)) * HX + (nn & 7); }

// out[b][o][v] = act(bias[o] + sum_{i,t} wp[i][t][o] in[b][i][v + t - 1]) with
// M = 16 output channels, N = the 256 voxels of an 8 x 8 x 4 tile (each wave
// 64 of them as four 16-voxel column blocks), K = input channel x tap.  The
// input halos and the matching weight slab are staged in LDS, double-buffered.
// grid (tiles, o_n / 16, batch).
template <bool RELU>
__global__ void __launch_bounds__(NT) conv3_mfma(const float* __restrict__ in, int i_n, const float* __restrict__ wp,
                                                 const float* __restrict__ bias, float* __restrict__ out, int o_n,
                                                 int R) {
  __shared__ float tile[2][CCH * HALO];
  __shared__ float ws[2][KST][MO];
  const TileIdx q = tile_of(blockIdx.x, R);
  const int o0 = blockIdx.y * MO, b = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ml = lane & 15, kq = lane >> 4;
  const int V = R * R * R;
  const float* src = in + (size_t)b * i_n * V;
  int bofs[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) bofs[nb] = voxel_offset(wave * 64 + nb * 16 + ml);
  v4f acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
  float pre[PF], prew[PW];
  auto wload = [&](int i0) {
#pragma unroll
    for (int k = 0; k < PW; ++k) {
      const int e = threadIdx.x + k * NT;
      float v = 0.f;
      if (e < KST * MO) {
        const int kk = e / MO, mm = e - kk * MO;
        const int i = i0 + kk / 27, t = kk % 27;
        if (i < i_n) v = wp[((size_t)i * 27 + t) * o_n + o0 + mm];
      }
      prew[k] = v;
    }
  };
  auto wstore = [&](int buf) {
#pragma unroll
    for (int k = 0; k < PW; ++k) {
      const int e = threadIdx.x + k * NT;
      if (e < KST * MO) ws[buf][e / MO][e % MO] = prew[k];
    }
  };
  halo_load(src, 0, i_n, R, q, pre);
  wload(0);
  halo_store(tile[0], pre);
  wstore(0);
  __syncthreads();
  const int nch = (i_n + CCH - 1) / CCH;
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more) {
      halo_load(src, (ch + 1) * CCH, i_n, R, q, pre);
      wload((ch + 1) * CCH);
    }
    const float* tl = tile[buf];
#pragma unroll 3
    for (int ks = 0; ks < KST; ks += 4) {
      const int k = ks + kq;
      const int cc = k / 27, t = k - cc * 27;
      const int toff = cc * HALO + tap_offset(t);
      const float a = ws[buf][k][ml];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, tl[toff + bofs[nb]], acc[nb], 0, 0, 0);
    }
    if (more) {
      halo_store(tile[buf ^ 1], pre);
      wstore(buf ^ 1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int nn = wave * 64 + nb * 16 + ml;
    const int x = q.x0 + (nn & 7), y = q.y0 + ((nn >> 3) & 7), z = q.z0 + (nn >> 6);
    if (x < R && y < R && z < R) {
      const int v = (z * R + y) * R + x;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = o0 + 4 * kq + e;
        float a = acc[nb][e] + (bias ? bias[o] : 0.f);
        if (RELU) a = a > 0.f ? a : 0.f;
        out[((size_t)b * o_n + o) * V + v] = a;
      }
    }
  }
}

// Weight and bias gradients as one GEMM per tile: D[o][(i, t)] += sum_v
// dout[b][o][v] X[(i, t)][v], M = 16 output channels, K = the tile's 256
// voxels, N = CCH input channels x 32 columns (27 taps, a column of ones that
// yields the bias gradient, padding).  Partial sums per slice of the
// (batch, tile) range: part[s][co][ci][t], bpart[s][co] (ci-chunk 0).
// grid (ci_n / CCH, co_n / 16, S).
__global__ void __launch_bounds__(NT) conv3_wgrad_mfma(const float* __restrict__ in, int ci_n,
                                                       const float* __restrict__ dout, int co_n, int batch, int R,
                                                       float* __restrict__ part, float* __restrict__ bpart) {
  __shared__ float tile[CCH * HALO];
  __shared__ float dts[MO][TX * TY * TZ + 4];
  const int i0 = blockIdx.x * CCH, o0 = blockIdx.y * MO, s = blockIdx.z, S = gridDim.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ml = lane & 15, kq = lane >> 4;
  const int V = R * R * R;
  const int nt = tiles_of(R);
  const int total = batch * nt;
  const int chunk = (total + S - 1) / S;
  const int e0 = s * chunk, e1 = min(total, e0 + chunk);
  // this lane's two B columns: n = (2 wave + j) 16 + ml -> channel cc, tap t
  int ncc[2], nt_[2], noff[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = (2 * wave + j) * 16 + ml;
    ncc[j] = n >> 5;
    nt_[j] = n & 31;
    noff[j] = ncc[j] * HALO + (nt_[j] < 27 ? tap_offset(nt_[j]) : 0);
  }
  v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
  for (int e = e0; e < e1; ++e) {
    const int b = e / nt;
    const TileIdx q = tile_of(e - b * nt, R);
    float pre[PF];
    halo_load(in + (size_t)b * ci_n * V, i0, ci_n, R, q, pre);
    // dout of the 16 output channels on the tile's voxels (0 outside the domain)
    float g[MO];
    {
      const int x = q.x0 + q.tx, y = q.y0 + q.ty, z = q.z0 + q.tz;
      const bool inside = x < R && y < R && z < R;
      const float* gp = dout + ((size_t)b * co_n + o0) * V + (size_t)((z * R + y) * R + x);
#pragma unroll
      for (int c = 0; c < MO; ++c) g[c] = inside ? gp[(size_t)c * V] : 0.f;
    }
    halo_store(tile, pre);
#pragma unroll
    for (int c = 0; c < MO; ++c) dts[c][threadIdx.x] = g[c];
    __syncthreads();
#pragma unroll 4
    for (int kv = 0; kv < TX * TY * TZ; kv += 4) {
      const int vx = kv + kq;
      const int vo = voxel_offset(vx);
      const float a = dts[ml][vx];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float bv = nt_[j] < 27 ? tile[noff[j] + vo] : (nt_[j] == 27 ? 1.f : 0.f);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int ci = i0 + ncc[j], t = nt_[j];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = o0 + 4 * kq + e;
      if (t < 27 && ci < ci_n) part[(((size_t)s * co_n + o) * ci_n + ci) * 27 + t] = acc[j][e];
      else if (t == 27 && ncc[j] == 0 && blockIdx.x == 0) bpart[(size_t)s * co_n + o] = acc[j][e];
    }
  }
}

// Packed copies of one 3x3x3 convolution's working weights w[co][ci][27]:
// wf[ci][t][co] = w[co][ci][t] (forward) and wb[co][t][ci] = w[co][ci][26 - t]
// (input gradient: the same GEMM with mirrored taps and channels swapped).
__global__ void repack3(const float* __restrict__ w, int ci_n, int co_n, float* __restrict__ wf,
                        float* __restrict__ wb) {
  const int n = co_n * ci_n * 27;
  for (int e = blockIdx.x * NT + threadIdx.x; e < n; e += gridDim.x * NT) {
    const int t = e % 27, ci = (e / 27) % ci_n, co = e / (27 * ci_n);
    wf[((size_t)ci * 27 + t) * co_n + co] = w[e];
    wb[((size_t)co * 27 + (26 - t)) * ci_n + ci] = w[e];
  }
}

// dw[j] = sum_s part[s][j] for j < len (fixed order over s)
__global__ void sum_slices(const float* __restrict__ part, int S, int64_t len, float* __restrict__ dw) {
  for (int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x; j < len; j += (int64_t)gridDim.x * NT) {
    float a = 0.f;
    for (int s = 0; s < S; ++s) a += part[(size_t)s * len + j];
    dw[j] = a;
  }
}

// ---- pooling, upsampling, skip connections, ReLU gradient ------------------------------
// g *= (y > 0): gradient through a ReLU whose output is y
__global__ void relu_bwd(const float* __restrict__ y, float* __restrict__ g, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
    if (!(y[e] > 0.f)) g[e] = 0.f;
}

// out[p][Z][Y][X] = mean of the 2x2x2 block of in[p] (p = batch*channel planes of R^3)
__global__ void pool_fwd(const float* __restrict__ in, float* __restrict__ out, int64_t planes, int R) {
  const int r = R / 2;
  const int64_t v3 = (int64_t)r * r * r, n = planes * v3;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const int64_t p = e / v3;
    const int v = (int)(e - p * v3);
    const int x = v % r, y = (v / r) % r, z = v / (r * r);
    const float* s = in + p * R * R * R + ((size_t)(2 * z) * R + 2 * y) * R + 2 * x;
    const float a = s[0] + s[1] + s[R] + s[R + 1] + s[R * R] + s[R * R + 1] + s[R * R + R] + s[R * R + R + 1];
    out[e] = 0.125f * a;
  }
}
// adjoint of pool_fwd: din (R^3 planes) = dout (of the parent block) / 8
__global__ void pool_bwd(const float* __restrict__ dout, float* __restrict__ din, int64_t planes, int R) {
  const int r = R / 2;
  const int64_t V = (int64_t)R * R * R, n = planes * V;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const int64_t p = e / V;
    const int v = (int)(e - p * V);
    const int x = v % R, y = (v / R) % R, z = v / (R * R);
    din[e] = 0.125f * dout[p * r * r * r + ((size_t)(z >> 1) * r + (y >> 1)) * r + (x >> 1)];
  }
}
// nearest 2x upsampling of in [batch][c_in][r^3] into channels [0, c_in) of out [batch][c_tot][(2r)^3]
__global__ void up_fwd(const float* __restrict__ in, int c_in, float* __restrict__ out, int c_tot, int batch,
                       int r) {
  const int R = 2 * r;
  const int64_t V = (int64_t)R * R * R, n = (int64_t)batch * c_in * V;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const int64_t bc = e / V;
    const int v = (int)(e - bc * V);
    const int c = (int)(bc % c_in), b = (int)(bc / c_in);
    const int x = v % R, y = (v / R) % R, z = v / (R * R);
    out[((size_t)b * c_tot + c) * V + v] =
        in[((size_t)b * c_in + c) * r * r * r + ((size_t)(z >> 1) * r + (y >> 1)) * r + (x >> 1)];
  }
}
// adjoint of up_fwd: din = sum of the 8 children in channels [0, c_in) of dout
__global__ void up_bwd(const float* __restrict__ dout, int c_tot, float* __restrict__ din, int c_in, int batch,
                       int r) {
  const int R = 2 * r;
  const int64_t v3 = (int64_t)r * r * r, n = (int64_t)batch * c_in * v3;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const int64_t bc = e / v3;
    const int v = (int)(e - bc * v3);
    const int c = (int)(bc % c_in), b = (int)(bc / c_in);
    const int x = v % r, y = (v / r) % r, z = v / (r * r);
    const float* s = dout + ((size_t)b * c_tot + c) * R * R * R + ((size_t)(2 * z) * R + 2 * y) * R + 2 * x;
    din[e] = s[0] + s[1] + s[R] + s[R + 1] + s[R * R] + s[R * R + 1] + s[R * R + R] + s[R * R + R + 1];
  }
}
// dst[b][d0 + c] (=|+=) src[b][s0 + c], c < c_n, planes of V voxels
template <bool ADD>
__global__ void slice_copy(const float* __restrict__ src, int s_tot, int s0, float* __restrict__ dst, int d_tot,
                           int d0, int c_n, int batch, int V) {
  const int64_t n = (int64_t)batch * c_n * V;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const int64_t bc = e / V;
    const int v = (int)(e - bc * V);
    const int c = (int)(bc % c_n), b = (int)(bc / c_n);
    const float s = src[((size_t)b * s_tot + s0 + c) * V + v];
    float* d = dst + ((size_t)b * d_tot + d0 + c) * V + v;
    if (ADD) *d += s;
    else *d = s;
  }
}

// ---- inputs, loss, optimizer -------------------------------------------------------
// in[b][0..2] = 2 * centre - 1 per axis, in[b][3] = normalized log10 Gr_b
__global__ void make_inputs(const double* __restrict__ cen, const double* __restrict__ lg, int batch, int R,
                            float* __restrict__ in) {
  const int V = R * R * R;
  const int64_t n = (int64_t)batch * V;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const int b = (int)(e / V), v = (int)(e - (int64_t)b * V);
    const int x = v % R, y = (v / R) % R, z = v / (R * R);
    float* o = in + (size_t)b * 4 * V + v;
    o[0] = (float)(2.0 * cen[x] - 1.0);
    o[V] = (float)(2.0 * cen[R + y] - 1.0);
    o[2 * (size_t)V] = (float)(2.0 * cen[2 * R + z] - 1.0);
    o[3 * (size_t)V] = (float)lg[b];
  }
}

// g = 2 (p - t) / n; block partial sums of (p - t)^2 in FP64
__global__ void __launch_bounds__(NT) mse(const float* __restrict__ p, const float* __restrict__ t,
                                          float* __restrict__ g, int64_t n, double* __restrict__ part) {
  __shared__ double red[NT / 64];
  double a = 0.0;
  const float sc = (float)(2.0 / (double)n);
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float d = p[e] - t[e];
    a += (double)d * d;
    g[e] = sc * d;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < NT / 64; ++k) s += red[k];
    part[blockIdx.x] = s;
  }
}
__global__ void mse_finish(const double* __restrict__ part, int nb, double inv_n, double* __restrict__ out) {
  __shared__ double red[NT];
  double a = 0.0;
  for (int k = threadIdx.x; k < nb; k += NT) a += part[k];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * inv_n;
}

// Adam on the FP32 master weights, then their BF16-rounded working copy.
// omb1 = 1 - beta1 and omb2 = 1 - beta2 come rounded from FP64: formed in
// FP32, 1 - 0.999f would be off by 1.3e-5 relative.
__global__ void adam(float* __restrict__ w, float* __restrict__ wq, const float* __restrict__ g,
                     float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1, float omb1,
                     float b2, float omb2, float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float ge = g[e];
    const float me = b1 * m[e] + omb1 * ge;
    const float ve = b2 * v[e] + omb2 * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float we = w[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    w[e] = we;
    wq[e] = bf16_round(we);
  }
}
__global__ void quantize(const float* __restrict__ w, float* __restrict__ wq, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
    wq[e] = bf16_round(w[e]);
}
__global__ void fill0(float* __restrict__ p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) p[e] = 0.f;
}

inline int tiles_of_host(int R) { return ((R + 7) / 8) * ((R + 7) / 8) * ((R + 3) / 4); }

inline unsigned nblk(int64_t n) {
  return (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (n + NT - 1) / NT));
}

struct Conv {
  int ci, co, ks;
  int64_t w_off, b_off;  // offsets in the parameter vector
};

// activations: encoder, pooled, decoder inputs (concatenations) and outputs
enum { E1A, E1, P1, E2A, E2, P2, E3A, E3, CAT4, D4A, D2, CAT5, D5A, D1, OUT, NACT };
constexpr int act_ch[NACT] = {16, 16, 16, 32, 32, 32, 64, 64, 96, 32, 32, 48, 16, 16, 4};
constexpr int act_div[NACT] = {1, 1, 2, 2, 2, 4, 4, 4, 2, 2, 2, 1, 1, 1, 1};
// (ci, co, kernel size) of the 11 convolutions, in parameter order
constexpr int conv_spec[11][3] = {{4, 16, 3},  {16, 16, 3}, {16, 32, 3}, {32, 32, 3}, {32, 64, 3}, {64, 64, 3},
                                  {96, 32, 3}, {32, 32, 3}, {48, 16, 3}, {16, 16, 3}, {16, 4, 1}};

constexpr int kWgtBlocks = 2048;  // target block count of a weight-gradient launch
constexpr int kWgtCob = 4;        // output channels per block of the weight gradient

}  // namespace

struct kvnn {
  int R = 0, batch_max = 0;
  hipStream_t stream = nullptr;
  double lg_mid = 0, lg_half = 1;
  std::vector<Conv> conv;
  int64_t nparam = 0;
  float *w = nullptr, *wq = nullptr, *gw = nullptr, *m = nullptr, *v = nullptr;
  int step = 0;
  float *act = nullptr, *grad = nullptr;
  std::vector<int64_t> off;
  float* wpart = nullptr;  // weight-gradient slice partials
  float* bpart = nullptr;  // bias-gradient slice partials
  float* wpk = nullptr;    // packed working weights of the 3x3x3 convolutions
  std::vector<int64_t> pk_off;  // per convolution: offset of wf (wb follows)
  double *cen = nullptr, *lg = nullptr, *part = nullptr, *loss = nullptr;
  float* in1 = nullptr;  // inputs of kvnn_predict
  std::string err;
};

namespace {

int fail(kvnn* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  return code;
}

#define NNCHK(n, call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fail((n), KVNN_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

float* A(kvnn* n, int k) { return n->act + n->off[k]; }
float* G(kvnn* n, int k) { return n->grad + n->off[k]; }

// voxel slices of a weight-gradient launch: enough blocks to fill the chip
int wgt_slices(const Conv& c) {
  const int blocks = c.ci * (c.co / kWgtCob);
  return std::max(1, std::min(64, kWgtBlocks / blocks));
}

// slices of a 3x3x3 weight-gradient launch: enough blocks to fill the chip
int wgrad3_slices(const Conv& c) {
  const int blocks = ((c.ci + CCH - 1) / CCH) * (c.co / MO);
  return std::max(1, std::min(64, kWgtBlocks / blocks));
}

hipError_t repack_all(kvnn* n) {
  for (size_t k = 0; k < n->conv.size(); ++k) {
    const Conv& c = n->conv[k];
    if (c.ks != 3) continue;
    const int64_t len = (int64_t)c.co * c.ci * 27;
    float* wf = n->wpk + n->pk_off[k];
    repack3<<<nblk(len), NT, 0, n->stream>>>(n->wq + c.w_off, c.ci, c.co, wf, wf + len);
  }
  return hipGetLastError();
}
int cob_of(const Conv& c) { return c.co % 8 == 0 ? 8 : 4; }
int cib_of(const Conv& c) { return c.ci % 8 == 0 ? 8 : 4; }

const float* packed_fwd(kvnn* n, const Conv& c) { return n->wpk + n->pk_off[&c - n->conv.data()]; }
const float* packed_bwd(kvnn* n, const Conv& c) {
  return packed_fwd(n, c) + (int64_t)c.co * c.ci * 27;
}

hipError_t conv_forward(kvnn* n, const Conv& c, const float* in, float* out, int batch, int R, bool relu) {
  const int V = R * R * R;
  if (c.ks == 3) {
    const dim3 grid(tiles_of_host(R), c.co / MO, batch);
    const float* b = n->wq + c.b_off;
    if (relu) conv3_mfma<true><<<grid, NT, 0, n->stream>>>(in, c.ci, packed_fwd(n, c), b, out, c.co, R);
    else conv3_mfma<false><<<grid, NT, 0, n->stream>>>(in, c.ci, packed_fwd(n, c), b, out, c.co, R);
    return hipGetLastError();
  }
  // the 1x1x1 head: one output voxel per lane, direct
  const int cob = cob_of(c);
  const dim3 grid((V + NT - 1) / NT, c.co / cob, batch);
  const float* w = n->wq + c.w_off;
  const float* b = n->wq + c.b_off;
#define KVNN_FWD(RL, CB) conv_fwd<1, RL, CB><<<grid, NT, 0, n->stream>>>(in, c.ci, w, b, out, c.co, R)
  if (cob == 8) {
    if (relu) KVNN_FWD(true, 8);
    else KVNN_FWD(false, 8);
  } else {
    if (relu) KVNN_FWD(true, 4);
    else KVNN_FWD(false, 4);
  }
#undef KVNN_FWD
  return hipGetLastError();
}

// gout: gradient with respect to the convolution output (after its ReLU
// mask); writes the parameter gradients and, when gin is not null, the input
// gradient.
hipError_t conv_backward(kvnn* n, const Conv& c, const float* in, const float* gout, float* gin, int batch, int R) {
  const int V = R * R * R;
  const int64_t wlen = (int64_t)c.co * c.ci * c.ks * c.ks * c.ks;
  if (c.ks == 3) {
    const int S = std::min(wgrad3_slices(c), batch * tiles_of_host(R));
    const dim3 wg((c.ci + CCH - 1) / CCH, c.co / MO, S);
    conv3_wgrad_mfma<<<wg, NT, 0, n->stream>>>(in, c.ci, gout, c.co, batch, R, n->wpart, n->bpart);
    sum_slices<<<nblk(wlen), NT, 0, n->stream>>>(n->wpart, S, wlen, n->gw + c.w_off);
    sum_slices<<<1, NT, 0, n->stream>>>(n->bpart, S, c.co, n->gw + c.b_off);
    if (gin) {
      const dim3 dg(tiles_of_host(R), c.ci / MO, batch);
      conv3_mfma<false><<<dg, NT, 0, n->stream>>>(gout, c.co, packed_bwd(n, c), nullptr, gin, c.ci, R);
    }
    return hipGetLastError();
  }
  const int S = wgt_slices(c);
  const dim3 wg(c.ci, c.co / kWgtCob, S);
  conv_bwd_weight<1, kWgtCob><<<wg, NT, 0, n->stream>>>(in, c.ci, gout, c.co, batch, R, n->wpart, n->bpart);
  sum_slices<<<nblk(wlen), NT, 0, n->stream>>>(n->wpart, S, wlen, n->gw + c.w_off);
  sum_slices<<<1, NT, 0, n->stream>>>(n->bpart, S, c.co, n->gw + c.b_off);
  if (gin) {
    const int cib = cib_of(c);
    const dim3 dg((V + NT - 1) / NT, c.ci / cib, batch);
    const float* w = n->wq + c.w_off;
    if (cib == 8) conv_bwd_data<1, 8><<<dg, NT, 0, n->stream>>>(gout, c.co, w, gin, c.ci, R);
    else conv_bwd_data<1, 4><<<dg, NT, 0, n->stream>>>(gout, c.co, w, gin, c.ci, R);
  }
  return hipGetLastError();
}

int forward(kvnn* n, const float* x, int batch) {
  const int R = n->R, r2 = R / 2, r4 = R / 4;
  const int V1 = R * R * R, V2 = r2 * r2 * r2, V4 = r4 * r4 * r4;
  const auto& C = n->conv;
  hipStream_t s = n->stream;
  NNCHK(n, conv_forward(n, C[0], x, A(n, E1A), batch, R, true));
  NNCHK(n, conv_forward(n, C[1], A(n, E1A), A(n, E1), batch, R, true));
  pool_fwd<<<nblk((int64_t)batch * 16 * V2), NT, 0, s>>>(A(n, E1), A(n, P1), (int64_t)batch * 16, R);
  NNCHK(n, conv_forward(n, C[2], A(n, P1), A(n, E2A), batch, r2, true));
  NNCHK(n, conv_forward(n, C[3], A(n, E2A), A(n, E2), batch, r2, true));
  pool_fwd<<<nblk((int64_t)batch * 32 * V4), NT, 0, s>>>(A(n, E2), A(n, P2), (int64_t)batch * 32, r2);
  NNCHK(n, conv_forward(n, C[4], A(n, P2), A(n, E3A), batch, r4, true));
  NNCHK(n, conv_forward(n, C[5], A(n, E3A), A(n, E3), batch, r4, true));
  up_fwd<<<nblk((int64_t)batch * 64 * V2), NT, 0, s>>>(A(n, E3), 64, A(n, CAT4), 96, batch, r4);
  slice_copy<false>
      <<<nblk((int64_t)batch * 32 * V2), NT, 0, s>>>(A(n, E2), 32, 0, A(n, CAT4), 96, 64, 32, batch, V2);
  NNCHK(n, conv_forward(n, C[6], A(n, CAT4), A(n, D4A), batch, r2, true));
  NNCHK(n, conv_forward(n, C[7], A(n, D4A), A(n, D2), batch, r2, true));
  up_fwd<<<nblk((int64_t)batch * 32 * V1), NT, 0, s>>>(A(n, D2), 32, A(n, CAT5), 48, batch, r2);
  slice_copy<false>
      <<<nblk((int64_t)batch * 16 * V1), NT, 0, s>>>(A(n, E1), 16, 0, A(n, CAT5), 48, 32, 16, batch, V1);
  NNCHK(n, conv_forward(n, C[8], A(n, CAT5), A(n, D5A), batch, R, true));
  NNCHK(n, conv_forward(n, C[9], A(n, D5A), A(n, D1), batch, R, true));
  NNCHK(n, conv_forward(n, C[10], A(n, D1), A(n, OUT), batch, R, false));
  return KVNN_OK;
}

// Gradient of the loss with respect to the output in G(OUT); parameter
// gradients overwrite n->gw.
int backward(kvnn* n, const float* x, int batch) {
  const int R = n->R, r2 = R / 2, r4 = R / 4;
  const int V1 = R * R * R, V2 = r2 * r2 * r2, V4 = r4 * r4 * r4;
  const auto& C = n->conv;
  hipStream_t s = n->stream;
  auto relu = [&](int k, int ch, int V) {
    const int64_t len = (int64_t)batch * ch * V;
    relu_bwd<<<nblk(len), NT, 0, s>>>(A(n, k), G(n, k), len);
  };
  NNCHK(n, conv_backward(n, C[10], A(n, D1), G(n, OUT), G(n, D1), batch, R));
  relu(D1, 16, V1);
  NNCHK(n, conv_backward(n, C[9], A(n, D5A), G(n, D1), G(n, D5A), batch, R));
  relu(D5A, 16, V1);
  NNCHK(n, conv_backward(n, C[8], A(n, CAT5), G(n, D5A), G(n, CAT5), batch, R));
  // CAT5 = [up(D2) (32) | E1 (16)]
  up_bwd<<<nblk((int64_t)batch * 32 * V2), NT, 0, s>>>(G(n, CAT5), 48, G(n, D2), 32, batch, r2);
  relu(D2, 32, V2);
  NNCHK(n, conv_backward(n, C[7], A(n, D4A), G(n, D2), G(n, D4A), batch, r2));
  relu(D4A, 32, V2);
  NNCHK(n, conv_backward(n, C[6], A(n, CAT4), G(n, D4A), G(n, CAT4), batch, r2));
  // CAT4 = [up(E3) (64) | E2 (32)]
  up_bwd<<<nblk((int64_t)batch * 64 * V4), NT, 0, s>>>(G(n, CAT4), 96, G(n, E3), 64, batch, r4);
  relu(E3, 64, V4);
  NNCHK(n, conv_backward(n, C[5], A(n, E3A), G(n, E3), G(n, E3A), batch, r4));
  relu(E3A, 64, V4);
  NNCHK(n, conv_backward(n, C[4], A(n, P2), G(n, E3A), G(n, P2), batch, r4));
  // E2 feeds the pooling and the skip connection
  pool_bwd<<<nblk((int64_t)batch * 32 * V2), NT, 0, s>>>(G(n, P2), G(n, E2), (int64_t)batch * 32, r2);
  slice_copy<true>
      <<<nblk((int64_t)batch * 32 * V2), NT, 0, s>>>(G(n, CAT4), 96, 64, G(n, E2), 32, 0, 32, batch, V2);
  relu(E2, 32, V2);
  NNCHK(n, conv_backward(n, C[3], A(n, E2A), G(n, E2), G(n, E2A), batch, r2));
  relu(E2A, 32, V2);
  NNCHK(n, conv_backward(n, C[2], A(n, P1), G(n, E2A), G(n, P1), batch, r2));
  pool_bwd<<<nblk((int64_t)batch * 16 * V1), NT, 0, s>>>(G(n, P1), G(n, E1), (int64_t)batch * 16, R);
  slice_copy<true>
      <<<nblk((int64_t)batch * 16 * V1), NT, 0, s>>>(G(n, CAT5), 48, 32, G(n, E1), 16, 0, 16, batch, V1);
  relu(E1, 16, V1);
  NNCHK(n, conv_backward(n, C[1], A(n, E1A), G(n, E1), G(n, E1A), batch, R));
  relu(E1A, 16, V1);
  NNCHK(n, conv_backward(n, C[0], x, G(n, E1A), nullptr, batch, R));
  return KVNN_OK;
}

int check_batch(kvnn* n, int batch) {
  if (batch < 1 || batch > n->batch_max) return fail(n, KVNN_EINVAL, "batch outside [1, batch_max]");
  return KVNN_OK;
}

}  // namespace

extern "C" {

int kvnn_create(const kvnn_params* p, void* hip_stream, kvnn** out) {
  if (!out) return KVNN_EINVAL;
  *out = nullptr;
  if (!p || p->res < 4 || p->res % 4 != 0 || p->res > 256 || p->batch_max < 1 || !p->xc || !p->yc || !p->zc ||
      !(p->lgr_hi > p->lgr_lo) || !std::isfinite(p->lgr_lo) || !std::isfinite(p->lgr_hi))
    return KVNN_EINVAL;
  const int R = p->res;
  // voxel indices are 32-bit: the largest activation of a batch must fit
  if ((int64_t)p->batch_max * 48 * R * R * R >= (int64_t(1) << 31)) return KVNN_EINVAL;
  std::vector<double> cen(3 * R);
  for (int i = 0; i < R; ++i) {
    cen[i] = p->xc[i];
    cen[R + i] = p->yc[i];
    cen[2 * R + i] = p->zc[i];
  }
  for (double c : cen)
    if (!(c >= 0.0 && c <= 1.0)) return KVNN_EINVAL;
  kvnn* n = new (std::nothrow) kvnn();
  if (!n) return KVNN_ENOMEM;
  n->R = R;
  n->batch_max = p->batch_max;
  n->stream = reinterpret_cast<hipStream_t>(hip_stream);
  n->lg_mid = 0.5 * (p->lgr_lo + p->lgr_hi);
  n->lg_half = 0.5 * (p->lgr_hi - p->lgr_lo);
  int64_t o = 0, wpart = 0, bpart = 0, pk = 0;
  for (const auto& s : conv_spec) {
    Conv c{s[0], s[1], s[2], 0, 0};
    const int64_t wl = (int64_t)c.co * c.ci * c.ks * c.ks * c.ks;
    c.w_off = o;
    c.b_off = o + wl;
    o += wl + c.co;
    const int sl = c.ks == 3 ? wgrad3_slices(c) : wgt_slices(c);
    wpart = std::max<int64_t>(wpart, wl * sl);
    bpart = std::max<int64_t>(bpart, (int64_t)c.co * sl);
    n->pk_off.push_back(pk);
    if (c.ks == 3) pk += 2 * wl;
    n->conv.push_back(c);
  }
  n->nparam = o;
  std::vector<float> w(o, 0.0f);
  std::mt19937_64 gen(p->seed);
  for (const auto& c : n->conv) {
    std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (c.ci * c.ks * c.ks * c.ks)));
    for (int64_t e = 0; e < c.b_off - c.w_off; ++e) w[c.w_off + e] = (float)nd(gen);
  }
  int64_t acc = 0;
  for (int k = 0; k < NACT; ++k) {
    n->off.push_back(acc);
    const int64_t r = R / act_div[k];
    acc += (int64_t)p->batch_max * act_ch[k] * r * r * r;
  }
  const int64_t V = (int64_t)R * R * R;
  auto bad = [&](int code) {
    kvnn_destroy(n);
    return code;
  };
  if (hipMalloc(&n->w, o * sizeof(float)) != hipSuccess || hipMalloc(&n->wq, o * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->gw, o * sizeof(float)) != hipSuccess || hipMalloc(&n->m, o * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->v, o * sizeof(float)) != hipSuccess || hipMalloc(&n->act, acc * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->grad, acc * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->wpart, wpart * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->bpart, bpart * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->wpk, pk * sizeof(float)) != hipSuccess ||
      hipMalloc(&n->cen, 3 * R * sizeof(double)) != hipSuccess ||
      hipMalloc(&n->lg, p->batch_max * sizeof(double)) != hipSuccess ||
      hipMalloc(&n->part, 8192 * sizeof(double)) != hipSuccess ||
      hipMalloc(&n->loss, sizeof(double)) != hipSuccess || hipMalloc(&n->in1, 4 * V * sizeof(float)) != hipSuccess)
    return bad(KVNN_ENOMEM);
  if (hipMemcpyAsync(n->w, w.data(), o * sizeof(float), hipMemcpyHostToDevice, n->stream) != hipSuccess ||
      hipMemcpyAsync(n->cen, cen.data(), 3 * R * sizeof(double), hipMemcpyHostToDevice, n->stream) != hipSuccess)
    return bad(KVNN_EDEVICE);
  fill0<<<nblk(o), NT, 0, n->stream>>>(n->m, o);
  fill0<<<nblk(o), NT, 0, n->stream>>>(n->v, o);
  quantize<<<nblk(o), NT, 0, n->stream>>>(n->w, n->wq, o);
  if (hipGetLastError() != hipSuccess || repack_all(n) != hipSuccess ||
      hipStreamSynchronize(n->stream) != hipSuccess)
    return bad(KVNN_EDEVICE);
  *out = n;
  return KVNN_OK;
}

int kvnn_destroy(kvnn* n) {
  if (!n) return KVNN_OK;
  if (n->w) hipStreamSynchronize(n->stream);
  for (void* p : {(void*)n->w, (void*)n->wq, (void*)n->gw, (void*)n->m, (void*)n->v, (void*)n->act, (void*)n->grad,
                  (void*)n->wpart, (void*)n->bpart, (void*)n->wpk, (void*)n->cen, (void*)n->lg, (void*)n->part, (void*)n->loss, (void*)n->in1})
    if (p) hipFree(p);
  delete n;
  return KVNN_OK;
}

int kvnn_num_params(const kvnn* n, int64_t* count) {
  if (!n || !count) return KVNN_EINVAL;
  *count = n->nparam;
  return KVNN_OK;
}

int kvnn_get_params(kvnn* n, float* host) {
  if (!n) return KVNN_EINVAL;
  if (!host) return fail(n, KVNN_EINVAL, "null output");
  NNCHK(n, hipMemcpyAsync(host, n->w, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  return KVNN_OK;
}

int kvnn_set_params(kvnn* n, const float* host) {
  if (!n) return KVNN_EINVAL;
  if (!host) return fail(n, KVNN_EINVAL, "null input");
  for (int64_t e = 0; e < n->nparam; ++e)
    if (!std::isfinite(host[e])) return fail(n, KVNN_EINVAL, "non-finite parameter");
  NNCHK(n, hipMemcpyAsync(n->w, host, n->nparam * sizeof(float), hipMemcpyHostToDevice, n->stream));
  quantize<<<nblk(n->nparam), NT, 0, n->stream>>>(n->w, n->wq, n->nparam);
  NNCHK(n, repack_all(n));
  fill0<<<nblk(n->nparam), NT, 0, n->stream>>>(n->m, n->nparam);
  fill0<<<nblk(n->nparam), NT, 0, n->stream>>>(n->v, n->nparam);
  NNCHK(n, hipGetLastError());
  NNCHK(n, hipStreamSynchronize(n->stream));
  n->step = 0;
  return KVNN_OK;
}

int kvnn_make_inputs(kvnn* n, const double* gr, int batch, float* in) {
  if (!n) return KVNN_EINVAL;
  if (!gr || !in) return fail(n, KVNN_EINVAL, "null argument");
  if (int rc = check_batch(n, batch)) return rc;
  std::vector<double> lg(batch);
  for (int b = 0; b < batch; ++b) {
    if (!(gr[b] > 0.0) || !std::isfinite(gr[b])) return fail(n, KVNN_EINVAL, "Gr must be positive and finite");
    lg[b] = (std::log10(gr[b]) - n->lg_mid) / n->lg_half;
  }
  NNCHK(n, hipMemcpyAsync(n->lg, lg.data(), batch * sizeof(double), hipMemcpyHostToDevice, n->stream));
  make_inputs<<<nblk((int64_t)batch * n->R * n->R * n->R), NT, 0, n->stream>>>(n->cen, n->lg, batch, n->R, in);
  NNCHK(n, hipGetLastError());
  // lg is a local host array: wait until its upload has completed
  NNCHK(n, hipStreamSynchronize(n->stream));
  return KVNN_OK;
}

int kvnn_forward(kvnn* n, const float* in, int batch, float* out) {
  if (!n) return KVNN_EINVAL;
  if (!in) return fail(n, KVNN_EINVAL, "null input");
  if (int rc = check_batch(n, batch)) return rc;
  if (int rc = forward(n, in, batch)) return rc;
  if (out) {
    const int64_t len = (int64_t)batch * 4 * n->R * n->R * n->R;
    NNCHK(n, hipMemcpyAsync(out, A(n, OUT), len * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
  }
  return KVNN_OK;
}

int kvnn_predict(kvnn* n, double Gr, float* out) {
  if (!n) return KVNN_EINVAL;
  if (int rc = kvnn_make_inputs(n, &Gr, 1, n->in1)) return rc;
  return kvnn_forward(n, n->in1, 1, out);
}

int kvnn_backward(kvnn* n, const float* in, const float* gout, int batch, float* grads_host) {
  if (!n) return KVNN_EINVAL;
  if (!in || !gout) return fail(n, KVNN_EINVAL, "null argument");
  if (int rc = check_batch(n, batch)) return rc;
  if (int rc = forward(n, in, batch)) return rc;
  const int64_t len = (int64_t)batch * 4 * n->R * n->R * n->R;
  NNCHK(n, hipMemcpyAsync(G(n, OUT), gout, len * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
  if (int rc = backward(n, in, batch)) return rc;
  if (grads_host)
    NNCHK(n, hipMemcpyAsync(grads_host, n->gw, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  return KVNN_OK;
}

int kvnn_train_step(kvnn* n, const float* in, const float* target, int batch, float lr, float* loss) {
  if (!n) return KVNN_EINVAL;
  if (!in || !target) return fail(n, KVNN_EINVAL, "null argument");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(n, KVNN_EINVAL, "learning rate must be positive");
  if (int rc = check_batch(n, batch)) return rc;
  if (int rc = forward(n, in, batch)) return rc;
  const int64_t len = (int64_t)batch * 4 * n->R * n->R * n->R;
  const unsigned nb = nblk(len);
  mse<<<nb, NT, 0, n->stream>>>(A(n, OUT), target, G(n, OUT), len, n->part);
  mse_finish<<<1, NT, 0, n->stream>>>(n->part, (int)nb, 1.0 / (double)len, n->loss);
  if (int rc = backward(n, in, batch)) return rc;
  ++n->step;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, n->step)), c2 = (float)(1.0 - std::pow(b2, n->step));
  adam<<<nblk(n->nparam), NT, 0, n->stream>>>(n->w, n->wq, n->gw, n->m, n->v, n->nparam, lr, (float)b1,
                                              (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), 1e-8f, c1, c2);
  NNCHK(n, hipGetLastError());
  NNCHK(n, repack_all(n));
  if (loss) {
    double h = 0.0;
    NNCHK(n, hipMemcpyAsync(&h, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    NNCHK(n, hipStreamSynchronize(n->stream));
    *loss = (float)h;
  }
  return KVNN_OK;
}

const char* kvnn_last_error(const kvnn* n) { return n ? n->err.c_str() : "kvnn: null handle"; }

}  // extern "C"
