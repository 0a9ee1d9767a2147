// Vector kernels of the Krylov solvers: volume-weighted inner products
// (single, fused pairs, and block Gram-Schmidt multi-dots), block updates,
// linear combinations and max-reductions.  All reductions are two-pass
// (per-block partials, then one finishing block) so results do not depend
// on scheduling.
//
// The weighted inner product walks the packed layout row by row: one wave
// per x-row, lanes along x, so every load is a coalesced row segment and the
// control volume of each unknown is the product of three per-axis metrics
// (never stored as a vector).
#include "kv_internal.h"

namespace kv {
namespace {

struct RowInfo {
  int64_t off;
  int len;
  const double* wx;
  double wyz;
};

// Row r of the packed vector: block u (nz*ny rows of nx-1), v (nz*(ny-1) rows
// of nx), w ((nz-1)*ny rows of nx), T (nz*ny rows of nx).
// (Row indices fit 32 bits: at most 4 * 4096^2 rows.)
__device__ __forceinline__ RowInfo row_info(const Grid& g, int64_t r64) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int R0 = nz * ny, R1 = nz * (ny - 1), R2 = (nz - 1) * ny;
  int r = (int)r64;
  if (r < R0) {
    const int k = r / ny, j = r - k * ny;
    return {g.ou + (int64_t)r * (nx - 1), nx - 1, g.ax[0].dd + 1, g.ax[1].h[j] * g.ax[2].h[k]};
  }
  r -= R0;
  if (r < R1) {
    const int k = r / (ny - 1), jj = r - k * (ny - 1);
    return {g.ov + (int64_t)r * nx, nx, g.ax[0].h, g.ax[1].dd[jj + 1] * g.ax[2].h[k]};
  }
  r -= R1;
  if (r < R2) {
    const int kk = r / ny, j = r - kk * ny;
    return {g.ow + (int64_t)r * nx, nx, g.ax[0].h, g.ax[1].h[j] * g.ax[2].dd[kk + 1]};
  }
  r -= R2;
  const int k = r / ny, j = r - k * ny;
  return {g.oT + (int64_t)r * nx, nx, g.ax[0].h, g.ax[1].h[j] * g.ax[2].h[k]};
}

__device__ __forceinline__ int64_t total_rows(const Grid& g) {
  return (int64_t)g.nz * g.ny * 2 + (int64_t)g.nz * (g.ny - 1) + (int64_t)(g.nz - 1) * g.ny;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of v over the 256-thread block (4 waves); valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  return (threadIdx.x == 0) ? (sh[0] + sh[1]) + (sh[2] + sh[3]) : 0.0;
}

struct Ptr4 {
  const double* p[4];
};

template <int NP>
__global__ void __launch_bounds__(256) wdots_kernel(Grid g, Ptr4 a, Ptr4 b, double* __restrict__ part) {
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = 0.0;
  const int64_t nrows = total_rows(g);
  for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < nrows; r += (int64_t)gridDim.x * 4) {
    const RowInfo ri = row_info(g, r);
    for (int e = lane; e < ri.len; e += 64) {
      const double w = ri.wx[e] * ri.wyz;
#pragma unroll
      for (int q = 0; q < NP; ++q) acc[q] += w * a.p[q][ri.off + e] * b.p[q][ri.off + e];
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const double s = block_sum(acc[q], sh);
    if (threadIdx.x == 0) part[(int64_t)q * gridDim.x + blockIdx.x] = s;
  }
}

// An empty asm that takes v[0..N) as register operands: every load that
// produced them is issued before this point.
template <int N>
__device__ __forceinline__ void hold_values(double* v) {
#pragma unroll
  for (int q = 0; q < N; ++q) asm volatile("" : "+v"(v[q]));
}

// Block sums of acc[0..NQ) over the 256-thread block with one barrier:
// wave sums into LDS, then thread q adds the four waves of value q (fixed
// order) and writes part[prow(q) * gridDim.x + blockIdx.x].
template <int NQ, typename RowOf>
__device__ __forceinline__ void block_sums(const double* acc, double* sh, double* __restrict__ part, RowOf prow) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) sh[wave * NQ + q] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NQ) {
    const int q = threadIdx.x;
    part[(int64_t)prow(q) * gridDim.x + blockIdx.x] = (sh[q] + sh[NQ + q]) + (sh[2 * NQ + q] + sh[3 * NQ + q]);
  }
}

// Block multi-dot for classical Gram-Schmidt: part[q][blk] for q < NV <= MD
// against the vectors V + q * ldv; w * weight is formed once per element.
// NV is a template parameter so that the NV loads of an element are issued
// together (a runtime count puts each behind its own branch).
constexpr int MD = 16;
template <int NV>
__global__ void __launch_bounds__(256) mdot_kernel(Grid g, const double* V, int64_t ldv,
                                                   const double* __restrict__ w, double* __restrict__ part,
                                                   int qbase) {
  __shared__ double sh[4 * NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  const int64_t nrows = total_rows(g);
  for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < nrows; r += (int64_t)gridDim.x * 4) {
    const RowInfo ri = row_info(g, r);
    for (int e = lane; e < ri.len; e += 64) {
      const int64_t idx = ri.off + e;
      double v[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = V[q * ldv + idx];
      double a = w[idx];
      const double wt = ri.wx[e] * ri.wyz;
      hold_values<NV>(v);
      asm volatile("" : "+v"(a));
      const double ww = wt * a;
#pragma unroll
      for (int q = 0; q < NV; ++q) acc[q] += ww * v[q];
    }
  }
  block_sums<NV>(acc, sh, part, [&](int q) { return qbase + q; });
}

// Two-vector block multi-dot of the delayed Gram-Schmidt: part[qbase + q]
// and part[ldp + qbase + q] for q < NV <= MD: <V_q, x1>_W and <V_q, x2>_W,
// each element of V read once for both.
template <int NV>
__global__ void __launch_bounds__(256) mdot2_kernel(Grid g, const double* V, int64_t ldv,
                                                    const double* __restrict__ x1, const double* __restrict__ x2,
                                                    double* __restrict__ part, int qbase, int ldp) {
  __shared__ double sh[4 * 2 * NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[2 * NV];  // x1 products, then x2 products
#pragma unroll
  for (int q = 0; q < 2 * NV; ++q) acc[q] = 0.0;
  const int64_t nrows = total_rows(g);
  for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < nrows; r += (int64_t)gridDim.x * 4) {
    const RowInfo ri = row_info(g, r);
    for (int e = lane; e < ri.len; e += 64) {
      const int64_t i0 = ri.off + e;
      // every load of the element is issued before the first product: the
      // empty asm takes the loaded values as operands, so all loads precede
      // it and one wait covers them (left alone, the scheduler keeps only
      // about four loads in flight, each next to its use)
      double v[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = V[q * ldv + i0];
      double a = x1[i0], b = x2[i0];
      const double wt = ri.wx[e] * ri.wyz;
      hold_values<NV>(v);
      asm volatile("" : "+v"(a), "+v"(b));
      const double u = wt * a, z = wt * b;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        acc[q] += u * v[q];
        acc[NV + q] += z * v[q];
      }
    }
  }
  block_sums<2 * NV>(acc, sh, part, [&](int q) { return q < NV ? qbase + q : ldp + qbase + (q - NV); });
}

// The fused update of the delayed Gram-Schmidt, one pass over V_0..V_{nv-1}:
//   w  <- cw w - cv v - sum_q d[q] V_q
//   v  <- cn (v - sum_q s[q] V_q)
// (d, s on the device, nv values each; nv may be 0).
__global__ void __launch_bounds__(256) mupdate2_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, int nv,
                                                       const double* __restrict__ d, const double* __restrict__ sv,
                                                       double cw, double cv, double cn, double* __restrict__ w,
                                                       double* __restrict__ v) {
  __shared__ double ds[512], ss[512];
  for (int q = threadIdx.x; q < nv; q += 256) {
    ds[q] = d[q];
    ss[q] = sv[q];
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double au = 0.0, av = 0.0;
    // (a two-buffer pipeline that keeps the next eight loads in flight
    // measured no faster at 256^3: 4.9 against 5.0 TB/s)
#pragma unroll 8
    for (int q = 0; q < nv; ++q) {
      const double x = V[q * ldv + e];
      au += ds[q] * x;
      av += ss[q] * x;
    }
    const double ve = v[e];
    w[e] = cw * w[e] - cv * ve - au;
    v[e] = cn * (ve - av);
  }
}

// out[q] = sum over blocks of part[q][blk]; one block per value q (the
// sums are independent; a single block looping over q made the finishing
// pass of a 200-vector multi-dot cost more than the multi-dot itself on
// small grids).
__global__ void __launch_bounds__(256) sum_finish_kernel(const double* __restrict__ part, int nblk,
                                                         double* __restrict__ out) {
  __shared__ double sh[4];
  const int q = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) v += part[(int64_t)q * nblk + b];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) out[q] = s;
}

// w -= sum_i h[i] V_i over the flat vector
__global__ void __launch_bounds__(256) mupdate_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, int nv,
                                                      const double* __restrict__ h, double* __restrict__ w) {
  __shared__ double hs[512];
  for (int q = threadIdx.x; q < nv; q += 256) hs[q] = h[q];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double acc = w[e];
    // eight loads in flight per thread
#pragma unroll 8
    for (int q = 0; q < nv; ++q) acc -= hs[q] * V[q * ldv + e];
    w[e] = acc;
  }
}

// out_q = sum_j W[j kq + q] V_j for q < kq <= KQ (a tall-skinny product V W
// of m vectors by an m x kq matrix).  Each thread owns one element index e:
// it reads V_j[e] for every j before writing out_q[e], so out may be V
// itself (ldo == ldv): the restart of a thick-restarted Arnoldi overwrites
// the first kq basis vectors in place.  W is read through scalar loads (its
// indices are uniform across the wave).
template <int KQ>
__global__ void __launch_bounds__(256) combine_kernel(int64_t n, const double* V, int64_t ldv, int m,
                                                      const double* __restrict__ W, int kq, double* out,
                                                      int64_t ldo) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double acc[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) acc[q] = 0.0;
    for (int j = 0; j < m; ++j) {
      const double v = V[j * ldv + e];
      const double* wj = W + (int64_t)j * kq;
#pragma unroll
      for (int q = 0; q < KQ; ++q)
        if (q < kq) acc[q] += wj[q] * v;
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q)
      if (q < kq) out[q * ldo + e] = acc[q];
  }
}

struct Coef4 {
  double c[4];
};

template <int NT>
__global__ void __launch_bounds__(256) lincomb_kernel(int64_t n, Coef4 c, Ptr4 in, double* out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double v = c.c[0] * in.p[0][e];
#pragma unroll
    for (int q = 1; q < NT; ++q) v += c.c[q] * in.p[q][e];
    out[e] = v;
  }
}

__global__ void __launch_bounds__(256) fill_kernel(int64_t n, double v, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) out[e] = v;
}

__device__ __forceinline__ double fin_abs(double v) {
  const double a = fabs(v);
  return (a <= 1.7976931348623157e308) ? a : __builtin_inf();
}

__global__ void __launch_bounds__(256) maxabs_kernel(int64_t n, const double* __restrict__ a, double* __restrict__ part) {
  __shared__ double s[256];
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    m = fmax(m, fin_abs(a[e]));
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void max1_finish_kernel(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  __shared__ double s[256];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) m = fmax(m, part[b]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

inline int flat_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

hipError_t launch_wdots(kv_ctx* c, int npair, const double* const* a, const double* const* b, double* out) {
  Ptr4 pa{}, pb{};
  for (int q = 0; q < npair; ++q) {
    pa.p[q] = a[q];
    pb.p[q] = b[q];
  }
  const int nblk = c->npart_blocks;
  switch (npair) {
    case 1: wdots_kernel<1><<<nblk, 256, 0, c->stream>>>(c->g, pa, pb, c->part); break;
    case 2: wdots_kernel<2><<<nblk, 256, 0, c->stream>>>(c->g, pa, pb, c->part); break;
    case 3: wdots_kernel<3><<<nblk, 256, 0, c->stream>>>(c->g, pa, pb, c->part); break;
    case 4: wdots_kernel<4><<<nblk, 256, 0, c->stream>>>(c->g, pa, pb, c->part); break;
    default: return hipErrorInvalidValue;
  }
  sum_finish_kernel<<<npair, 256, 0, c->stream>>>(c->part, nblk, out ? out : c->dres);
  return hipGetLastError();
}

// mdot_kernel<nv> / mdot2_kernel<nv> for a runtime nv in 1..MD
#define KV_MD_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_mdot(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* w, double* out) {
  if (nvec < 1 || nvec > 512) return hipErrorInvalidValue;
  const int nblk = c->nmd_blocks;
  for (int q0 = 0; q0 < nvec; q0 += MD) {
    const int nv = (nvec - q0 < MD) ? nvec - q0 : MD;
    const double* Vq = V + q0 * ldv;
    switch (nv) {
#define KV_MD1(N) \
  case N: mdot_kernel<N><<<nblk, 256, 0, c->stream>>>(c->g, Vq, ldv, w, c->part, q0); break;
      KV_MD_CASES(KV_MD1)
#undef KV_MD1
      default: return hipErrorInvalidValue;
    }
  }
  sum_finish_kernel<<<nvec, 256, 0, c->stream>>>(c->part, nblk, out ? out : c->dres);
  return hipGetLastError();
}

hipError_t launch_mdot2(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* x1, const double* x2,
                       double* out1, double* out2) {
  if (nvec < 1 || nvec > 512) return hipErrorInvalidValue;
  const int nblk = c->nmd_blocks;
  // partials: [q][blk] for x1 at rows q < nvec, for x2 at rows 512 + q
  for (int q0 = 0; q0 < nvec; q0 += MD) {
    const int nv = (nvec - q0 < MD) ? nvec - q0 : MD;
    const double* Vq = V + q0 * ldv;
    switch (nv) {
#define KV_MD2(N) \
  case N: mdot2_kernel<N><<<nblk, 256, 0, c->stream>>>(c->g, Vq, ldv, x1, x2, c->part, q0, 512); break;
      KV_MD_CASES(KV_MD2)
#undef KV_MD2
      default: return hipErrorInvalidValue;
    }
  }
  sum_finish_kernel<<<nvec, 256, 0, c->stream>>>(c->part, nblk, out1);
  sum_finish_kernel<<<nvec, 256, 0, c->stream>>>(c->part + (int64_t)512 * nblk, nblk, out2);
  return hipGetLastError();
}

hipError_t launch_mupdate2(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* d, const double* sv,
                           double cw, double cv, double cn, double* w, double* v) {
  if (nvec < 0 || nvec > 512) return hipErrorInvalidValue;
  mupdate2_kernel<<<flat_blocks(c->g.n), 256, 0, c->stream>>>(c->g.n, V, ldv, nvec, d, sv, cw, cv, cn, w, v);
  return hipGetLastError();
}

hipError_t launch_mupdate(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* h, double* w) {
  if (nvec < 1 || nvec > 512) return hipErrorInvalidValue;
  mupdate_kernel<<<flat_blocks(c->g.n), 256, 0, c->stream>>>(c->g.n, V, ldv, nvec, h, w);
  return hipGetLastError();
}

hipError_t launch_combine(const kv_ctx* c, const double* V, int64_t ldv, int m, const double* W, int kq,
                          double* out, int64_t ldo) {
  if (m < 1 || kq < 1 || kq > 64) return hipErrorInvalidValue;
  const int64_t n = c->g.n;
  const int nb = flat_blocks(n);
  if (kq <= 8) combine_kernel<8><<<nb, 256, 0, c->stream>>>(n, V, ldv, m, W, kq, out, ldo);
  else if (kq <= 16) combine_kernel<16><<<nb, 256, 0, c->stream>>>(n, V, ldv, m, W, kq, out, ldo);
  else if (kq <= 32) combine_kernel<32><<<nb, 256, 0, c->stream>>>(n, V, ldv, m, W, kq, out, ldo);
  else combine_kernel<64><<<nb, 256, 0, c->stream>>>(n, V, ldv, m, W, kq, out, ldo);
  return hipGetLastError();
}

hipError_t launch_lincomb(const kv_ctx* c, int64_t n, int nterm, const double* coef, const double* const* in,
                          double* out) {
  Coef4 cf{};
  Ptr4 p{};
  for (int q = 0; q < nterm; ++q) {
    cf.c[q] = coef[q];
    p.p[q] = in[q];
  }
  const int nb = flat_blocks(n);
  switch (nterm) {
    case 1: lincomb_kernel<1><<<nb, 256, 0, c->stream>>>(n, cf, p, out); break;
    case 2: lincomb_kernel<2><<<nb, 256, 0, c->stream>>>(n, cf, p, out); break;
    case 3: lincomb_kernel<3><<<nb, 256, 0, c->stream>>>(n, cf, p, out); break;
    case 4: lincomb_kernel<4><<<nb, 256, 0, c->stream>>>(n, cf, p, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill(const kv_ctx* c, int64_t n, double v, double* out) {
  fill_kernel<<<flat_blocks(n), 256, 0, c->stream>>>(n, v, out);
  return hipGetLastError();
}

hipError_t launch_maxabs(kv_ctx* c, const double* a, int64_t n) {
  const int nblk = c->npart_blocks;
  maxabs_kernel<<<nblk, 256, 0, c->stream>>>(n, a, c->part);
  max1_finish_kernel<<<1, 256, 0, c->stream>>>(c->part, nblk, c->dres);
  return hipGetLastError();
}

}  // namespace kv
