// The steady-state predictor of kvnn.h: a three-level 3-D U-Net trained by
// hand-written forward and backward kernels.  Convolutions are direct (one
// output voxel per lane, several output channels per lane so every loaded
// input value feeds several FMAs); their weights are the BF16-rounded master
// weights, products are accumulated in FP32.  Reductions (weight and bias
// gradients, the loss) are computed in a fixed order, so results do not
// depend on scheduling.
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
                                                      float* __restrict__ part) {
  constexpr int T = KS * KS * KS, H = KS / 2;
  __shared__ float red[NT / 64][COB * T];
  const int ci = blockIdx.x, co0 = blockIdx.y * COB, s = blockIdx.z, S = gridDim.z;
  const int V = R * R * R;
  const int total = batch * V;
  const int chunk = (total + S - 1) / S;
  const int e0 = s * chunk, e1 = min(total, e0 + chunk);
  float acc[COB][T];
#pragma unroll
  for (int c = 0; c < COB; ++c)
#pragma unroll
    for (int t = 0; t < T; ++t) acc[c][t] = 0.f;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += NT) {
    const int b = e / V, v = e - b * V;
    const int x = v % R, y = (v / R) % R, z = v / (R * R);
    float g[COB];
#pragma unroll
    for (int c = 0; c < COB; ++c) g[c] = dout[((size_t)b * co_n + co0 + c) * V + v];
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
  // wave sums (butterfly), then the waves in order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < COB; ++c)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      float a = acc[c][t];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      if (lane == 0) red[wv][c * T + t] = a;
    }
  __syncthreads();
  for (int q = threadIdx.x; q < COB * T; q += NT) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) a += red[k][q];
    const int c = q / T, t = q - c * T;
    part[(((size_t)s * co_n + co0 + c) * ci_n + ci) * T + t] = a;
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

// db[co] = sum_b sum_v dout[b][co][v]; one block per co
__global__ void __launch_bounds__(NT) bias_grad(const float* __restrict__ dout, int co_n, int batch, int V,
                                                float* __restrict__ db) {
  __shared__ float red[NT / 64];
  const int co = blockIdx.x;
  float a = 0.f;
  for (int b = 0; b < batch; ++b) {
    const float* g = dout + ((size_t)b * co_n + co) * V;
    for (int v = threadIdx.x; v < V; v += NT) a += g[v];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int k = 0; k < NT / 64; ++k) s += red[k];
    db[co] = s;
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
int cob_of(const Conv& c) { return c.co % 8 == 0 ? 8 : 4; }
int cib_of(const Conv& c) { return c.ci % 8 == 0 ? 8 : 4; }

hipError_t conv_forward(kvnn* n, const Conv& c, const float* in, float* out, int batch, int R, bool relu) {
  const int V = R * R * R;
  const int cob = cob_of(c);
  const dim3 grid((V + NT - 1) / NT, c.co / cob, batch);
  const float* w = n->wq + c.w_off;
  const float* b = n->wq + c.b_off;
#define KVNN_FWD(KS, RL, CB) conv_fwd<KS, RL, CB><<<grid, NT, 0, n->stream>>>(in, c.ci, w, b, out, c.co, R)
  if (c.ks == 3) {
    if (cob == 8) {
      if (relu) KVNN_FWD(3, true, 8);
      else KVNN_FWD(3, false, 8);
    } else {
      if (relu) KVNN_FWD(3, true, 4);
      else KVNN_FWD(3, false, 4);
    }
  } else {
    if (cob == 8) {
      if (relu) KVNN_FWD(1, true, 8);
      else KVNN_FWD(1, false, 8);
    } else {
      if (relu) KVNN_FWD(1, true, 4);
      else KVNN_FWD(1, false, 4);
    }
  }
#undef KVNN_FWD
  return hipGetLastError();
}

// gout: gradient with respect to the convolution output (after its ReLU
// mask); writes the parameter gradients and, when gin is not null, the input
// gradient.
hipError_t conv_backward(kvnn* n, const Conv& c, const float* in, const float* gout, float* gin, int batch, int R) {
  const int V = R * R * R;
  const int S = wgt_slices(c);
  const dim3 wg(c.ci, c.co / kWgtCob, S);
  if (c.ks == 3) conv_bwd_weight<3, kWgtCob><<<wg, NT, 0, n->stream>>>(in, c.ci, gout, c.co, batch, R, n->wpart);
  else conv_bwd_weight<1, kWgtCob><<<wg, NT, 0, n->stream>>>(in, c.ci, gout, c.co, batch, R, n->wpart);
  const int64_t wlen = (int64_t)c.co * c.ci * c.ks * c.ks * c.ks;
  sum_slices<<<nblk(wlen), NT, 0, n->stream>>>(n->wpart, S, wlen, n->gw + c.w_off);
  bias_grad<<<c.co, NT, 0, n->stream>>>(gout, c.co, batch, V, n->gw + c.b_off);
  if (gin) {
    const int cib = cib_of(c);
    const dim3 dg((V + NT - 1) / NT, c.ci / cib, batch);
    const float* w = n->wq + c.w_off;
    if (c.ks == 3) {
      if (cib == 8) conv_bwd_data<3, 8><<<dg, NT, 0, n->stream>>>(gout, c.co, w, gin, c.ci, R);
      else conv_bwd_data<3, 4><<<dg, NT, 0, n->stream>>>(gout, c.co, w, gin, c.ci, R);
    } else {
      if (cib == 8) conv_bwd_data<1, 8><<<dg, NT, 0, n->stream>>>(gout, c.co, w, gin, c.ci, R);
      else conv_bwd_data<1, 4><<<dg, NT, 0, n->stream>>>(gout, c.co, w, gin, c.ci, R);
    }
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
  int64_t o = 0, wpart = 0;
  for (const auto& s : conv_spec) {
    Conv c{s[0], s[1], s[2], 0, 0};
    const int64_t wl = (int64_t)c.co * c.ci * c.ks * c.ks * c.ks;
    c.w_off = o;
    c.b_off = o + wl;
    o += wl + c.co;
    wpart = std::max<int64_t>(wpart, wl * wgt_slices(c));
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
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess) return bad(KVNN_EDEVICE);
  *out = n;
  return KVNN_OK;
}

int kvnn_destroy(kvnn* n) {
  if (!n) return KVNN_OK;
  if (n->w) hipStreamSynchronize(n->stream);
  for (void* p : {(void*)n->w, (void*)n->wq, (void*)n->gw, (void*)n->m, (void*)n->v, (void*)n->act, (void*)n->grad,
                  (void*)n->wpart, (void*)n->cen, (void*)n->lg, (void*)n->part, (void*)n->loss, (void*)n->in1})
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
