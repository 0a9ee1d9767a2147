// Even/odd split of the fast-diagonalization transforms for mirror-symmetric
// axes (h_i = h_{N-1-i}, N even; both grids of the workloads are).
//
// A persymmetric M has eigenvectors that are either symmetric or
// antisymmetric about the midpoint, q = [w; +-J w] / sqrt(2), with w the
// eigenvectors of the half-size matrices M_11 +- M_{H-1,H} e e^T (H = N/2).
// The transform of f along the axis then needs only half-size products:
//   forward:  c_even = Qe^T (f_lo + J f_hi),  c_odd = Qo^T (f_lo - J f_hi)
//   inverse:  t = Qe c_even, u = Qo c_odd,   f_lo = t + u, J f_hi = t - u
// (Qe, Qo hold the first halves of the full unit eigenvectors), i.e. 6N
// instead of 12N flop per cell for the three axes of one Poisson solve.  The
// butterflies are fused into the operand loads (forward) and the epilogue
// (inverse); every product runs on v_mfma_f64_16x16x4.
//
// Coefficient order along a split axis: [H even modes | H odd modes].
#include <cstdlib>

#include "kv_internal.h"

namespace kv {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Storage / matrix-core precision of one transform pass.  FP64:
// v_mfma_f64_16x16x4 (D[i][j] in lane j + 16 (i % 4), element i / 4).  FP32:
// v_mfma_f32_16x16x4 (D[i][j] in lane j + 16 (i / 4), element i % 4), the
// mixed form's transforms.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

enum { RIGHT_FWD = 0, RIGHT_INV = 1, LEFT_FWD = 2, LEFT_INV = 3 };
enum { EPI_NONE = 0, EPI_DIVIDE = 1, EPI_ISQ = 2 };

struct SplitEpi {
  const double *lx, *ly, *lz;
  const double *isx, *isy, *isz;
  int nx, ny;
  int64_t null3;
};

constexpr int OOB = 0x7ffffff8;  // a byte offset past every buffer: raw buffer loads return 0

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const T* p, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, (int)(n * (int64_t)sizeof(T)), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int off);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Two consecutive elements in one load (16 bytes for FP64, 8 for FP32).
template <typename T>
__device__ __forceinline__ void bload2(__amdgpu_buffer_rsrc_t r, int off, T& x0, T& x1);
// (Elements are copied to scalars before the bit cast: a bit cast applied
// to a vector element directly reads element 0 whatever the index.)
template <>
__device__ __forceinline__ void bload2<double>(__amdgpu_buffer_rsrc_t r, int off, double& x0, double& x1) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  const unsigned long long w0 = (unsigned long long)v[0] | ((unsigned long long)v[1] << 32);
  const unsigned long long w1 = (unsigned long long)v[2] | ((unsigned long long)v[3] << 32);
  x0 = __builtin_bit_cast(double, w0);
  x1 = __builtin_bit_cast(double, w1);
}
template <>
__device__ __forceinline__ void bload2<float>(__amdgpu_buffer_rsrc_t r, int off, float& x0, float& x1) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  const unsigned w0 = v[0], w1 = v[1];
  x0 = __builtin_bit_cast(float, w0);
  x1 = __builtin_bit_cast(float, w1);
}

template <typename T>
struct SplitArgs {
  const T* in;
  T* out;
  const T* Qs;   // [2][H][H]: Qs[par][k][e]
  const T* QsT;  // [2][H][H]: QsT[par][e][k]
  int N, H;
  int64_t P;          // LEFT: contiguous length of a line (plane or row); RIGHT: unused
  int64_t R;          // RIGHT: number of rows; LEFT: unused
  int64_t bstride;    // LEFT: batch stride (y pass); 0 otherwise
  int batch;
  int mtiles, ntiles;
};

// One BM x BN output tile (4 waves in a 2 x 2 layout, each wave a
// (BM/2) x (BN/2) block of 16x16 MFMA accumulators).  RIGHT kinds: m = row, n = mode (fwd) or position
// (inv).  LEFT kinds: m = mode (fwd) or position (inv), n = line position p.
// The inverse kinds keep two accumulator sets (even -> t, odd -> u).
//
// VEC (every dimension the pairs run along is even: H, and the line length
// of the LEFT kinds): operands move in element pairs, A along k and B along n,
// so that the 64 lanes of one load cover whole contiguous row segments.
//
// Waves per SIMD the compiler must fit: 4 for the 64 x 64 inverse tiles (128
// VGPRs; left alone it takes 154 and runs 3, and 4 measured 3-5% faster per
// pass), 2 for the 128 x 128 forward tiles (the LDS holds two such blocks per
// CU), no constraint otherwise.
constexpr int split_waves(int kind, int bm, int bn) {
  return ((kind == 1 || kind == 3) && bm == 64 && bn == 64) ? 4 : ((bm == 128 && bn == 128) ? 2 : 1);
}

template <typename T, int KIND, int EPI, int BM, int BN, int BK, bool VEC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(split_waves(KIND, BM, BN))))
fd_split_kernel(SplitArgs<T> a, SplitEpi ep) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr bool INV = (KIND == RIGHT_INV || KIND == LEFT_INV);
  constexpr bool RIGHT = (KIND == RIGHT_FWD || KIND == RIGHT_INV);
  constexpr int NS = INV ? 2 : 1;  // operand sets
  constexpr int RM = BM / 32, RN = BN / 32;   // 16x16 blocks per wave
  constexpr int AE = BM * BK / 256, BE = BK * BN / 256;  // tile elements per thread
  // forward kinds double-buffer the LDS chunks (one barrier per chunk); the
  // inverse kinds carry two operand sets and keep one buffer (two barriers)
  constexpr int NB = INV ? 1 : 2;
  __shared__ T As[NB][NS][BK][BM + 2];
  __shared__ T Bs[NB][NS][BK][BN + 2];

  const int pars = INV ? 1 : 2;
  const int64_t total = (int64_t)a.mtiles * a.ntiles * a.batch * pars;
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t w = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (w >= total) return;
  // tile order: the tiles that share a big-operand tile are adjacent
  int mt, nt, par;
  int64_t b;
  {
    int64_t t = w;
    if (RIGHT) {  // big operand = rows (m); modes (n) and parity fastest
      par = (int)(t % pars);
      t /= pars;
      nt = (int)(t % a.ntiles);
      t /= a.ntiles;
      mt = (int)(t % a.mtiles);
      t /= a.mtiles;
    } else {      // big operand = line positions (n); modes (m) and parity fastest
      par = (int)(t % pars);
      t /= pars;
      mt = (int)(t % a.mtiles);
      t /= a.mtiles;
      nt = (int)(t % a.ntiles);
      t /= a.ntiles;
    }
    b = t;
  }
  if (INV) par = 0;
  const int N = a.N, H = a.H;
  const T sgn = par ? T(-1) : T(1);
  T* out = a.out + (RIGHT ? 0 : b * a.bstride);
  const int M = RIGHT ? (int)a.R : H;                 // rows of the output tile space
  const int64_t NN = RIGHT ? H : a.P;                 // columns of the output tile space
  const int K = H;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = mt * BM;
  const int64_t n0 = (int64_t)nt * BN;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  // A tile (BM x BK): thread -> row tid / (BK/AE'), AE consecutive k
  constexpr int AKT = BK / AE;                      // threads per A row
  const int ar = tid / AKT, ak = (tid % AKT) * AE;
  constexpr int BNT = BN / BE;                      // threads per B row
  const int bk = tid / BNT, bn = (tid % BNT) * BE;

  // Operand prefetch: raw buffer loads with 32-bit byte offsets (an offset
  // past the buffer reads 0, so edges need no branch and no load waits
  // inside the prefetch); the butterfly partner of a forward operand is
  // fetched separately and combined when the chunk is stashed into LDS.
  constexpr bool AFLY = (KIND == RIGHT_FWD), BFLY = (KIND == LEFT_FWD);
  const int64_t in_elems = RIGHT ? a.R * (int64_t)N : (int64_t)a.batch * a.bstride + (a.batch == 1 ? (int64_t)N * a.P : 0);
  const __amdgpu_buffer_rsrc_t rin = make_rsrc(a.in, in_elems);
  const __amdgpu_buffer_rsrc_t rq = make_rsrc(a.Qs, 2 * (int64_t)H * H);
  const __amdgpu_buffer_rsrc_t rqt = make_rsrc(a.QsT, 2 * (int64_t)H * H);
  const int64_t boff = RIGHT ? 0 : b * a.bstride;  // batch offset of a LEFT line block
  T ra[NS][AE], rb[NS][BE];
  T rah[AFLY ? NS : 1][AFLY ? AE : 1], rbh[BFLY ? NS : 1][BFLY ? BE : 1];
  auto fetch_one = [&](int k0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int ps = INV ? s : par;  // parity of this operand set
#pragma unroll
      for (int q = 0; q < AE; ++q) {
        const int gm = m0 + ar, gk = k0 + ak + q;
        const bool ok = gm < M && gk < K;
        int o = OOB, oh = OOB;
        if (KIND == RIGHT_FWD) {
          o = ok ? (gm * N + gk) * (int)sizeof(T) : OOB;
          oh = ok ? (gm * N + N - 1 - gk) * (int)sizeof(T) : OOB;
        } else if (KIND == RIGHT_INV) {
          o = ok ? (gm * N + ps * H + gk) * (int)sizeof(T) : OOB;
        } else {
          o = ok ? ((ps * H + gm) * H + gk) * (int)sizeof(T) : OOB;
        }
        if (KIND == RIGHT_FWD || KIND == RIGHT_INV) ra[s][q] = bload<T>(rin, o);
        else if (KIND == LEFT_FWD) ra[s][q] = bload<T>(rqt, o);
        else ra[s][q] = bload<T>(rq, o);
        if (AFLY) rah[AFLY ? s : 0][AFLY ? q : 0] = bload<T>(rin, oh);
      }
#pragma unroll
      for (int q = 0; q < BE; ++q) {
        const int gk = k0 + bk;
        const int64_t gn = n0 + bn + q;
        const bool ok = gk < K && gn < NN;
        int o = OOB, oh = OOB;
        if (KIND == RIGHT_FWD || KIND == RIGHT_INV) {
          o = ok ? ((ps * H + gk) * H + (int)gn) * (int)sizeof(T) : OOB;
          rb[s][q] = bload<T>(KIND == RIGHT_FWD ? rq : rqt, o);
        } else if (KIND == LEFT_FWD) {
          o = ok ? (int)((boff + (int64_t)gk * a.P + gn) * (int64_t)sizeof(T)) : OOB;
          oh = ok ? (int)((boff + (int64_t)(N - 1 - gk) * a.P + gn) * (int64_t)sizeof(T)) : OOB;
          rb[s][q] = bload<T>(rin, o);
          rbh[BFLY ? s : 0][BFLY ? q : 0] = bload<T>(rin, oh);
        } else {
          o = ok ? (int)((boff + (int64_t)(ps * H + gk) * a.P + gn) * (int64_t)sizeof(T)) : OOB;
          rb[s][q] = bload<T>(rin, o);
        }
      }
    }
  };
  // pair mapping (VEC): A pair p = tid + 256 h is row p / (BK/2), k 2 (p % (BK/2));
  // B pair p is row p / (BN/2), n 2 (p % (BN/2))
  constexpr int AKP = BK / 2, BNP = BN / 2;
  auto fetch_vec = [&](int k0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int ps = INV ? s : par;
#pragma unroll
      for (int h = 0; h < AE / 2; ++h) {
        const int pp = tid + 256 * h;
        const int gm = m0 + pp / AKP, gk = k0 + 2 * (pp % AKP);
        const bool ok = gm < M && gk < K;
        int o = OOB, oh = OOB;
        if (KIND == RIGHT_FWD) {
          o = ok ? (gm * N + gk) * (int)sizeof(T) : OOB;
          oh = ok ? (gm * N + N - 2 - gk) * (int)sizeof(T) : OOB;  // holds partners of gk + 1, gk
        } else if (KIND == RIGHT_INV) {
          o = ok ? (gm * N + ps * H + gk) * (int)sizeof(T) : OOB;
        } else {
          o = ok ? ((ps * H + gm) * H + gk) * (int)sizeof(T) : OOB;
        }
        const __amdgpu_buffer_rsrc_t r = (KIND == RIGHT_FWD || KIND == RIGHT_INV) ? rin : (KIND == LEFT_FWD ? rqt : rq);
        bload2<T>(r, o, ra[s][2 * h], ra[s][2 * h + 1]);
        if (AFLY) bload2<T>(rin, oh, rah[AFLY ? s : 0][AFLY ? 2 * h + 1 : 0], rah[AFLY ? s : 0][AFLY ? 2 * h : 0]);
      }
#pragma unroll
      for (int h = 0; h < BE / 2; ++h) {
        const int pp = tid + 256 * h;
        const int gk = k0 + pp / BNP;
        const int64_t gn = n0 + 2 * (pp % BNP);
        const bool ok = gk < K && gn < NN;
        int o = OOB, oh = OOB;
        if (KIND == RIGHT_FWD || KIND == RIGHT_INV) {
          o = ok ? ((ps * H + gk) * H + (int)gn) * (int)sizeof(T) : OOB;
          bload2<T>(KIND == RIGHT_FWD ? rq : rqt, o, rb[s][2 * h], rb[s][2 * h + 1]);
        } else if (KIND == LEFT_FWD) {
          o = ok ? (int)((boff + (int64_t)gk * a.P + gn) * (int64_t)sizeof(T)) : OOB;
          oh = ok ? (int)((boff + (int64_t)(N - 1 - gk) * a.P + gn) * (int64_t)sizeof(T)) : OOB;
          bload2<T>(rin, o, rb[s][2 * h], rb[s][2 * h + 1]);
          bload2<T>(rin, oh, rbh[BFLY ? s : 0][BFLY ? 2 * h : 0], rbh[BFLY ? s : 0][BFLY ? 2 * h + 1 : 0]);
        } else {
          o = ok ? (int)((boff + (int64_t)(ps * H + gk) * a.P + gn) * (int64_t)sizeof(T)) : OOB;
          bload2<T>(rin, o, rb[s][2 * h], rb[s][2 * h + 1]);
        }
      }
    }
  };
  auto stash_vec = [&](int buf) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int h = 0; h < AE / 2; ++h) {
        const int pp = tid + 256 * h;
        const int r = pp / AKP, k = 2 * (pp % AKP);
#pragma unroll
        for (int e = 0; e < 2; ++e)
          As[buf][s][k + e][r] = AFLY ? ra[s][2 * h + e] + sgn * rah[AFLY ? s : 0][AFLY ? 2 * h + e : 0] : ra[s][2 * h + e];
      }
#pragma unroll
      for (int h = 0; h < BE / 2; ++h) {
        const int pp = tid + 256 * h;
        const int k = pp / BNP, n = 2 * (pp % BNP);
#pragma unroll
        for (int e = 0; e < 2; ++e)
          Bs[buf][s][k][n + e] = BFLY ? rb[s][2 * h + e] + sgn * rbh[BFLY ? s : 0][BFLY ? 2 * h + e : 0] : rb[s][2 * h + e];
      }
    }
  };
  auto stash_one = [&](int buf) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int q = 0; q < AE; ++q)
        As[buf][s][ak + q][ar] = AFLY ? ra[s][q] + sgn * rah[AFLY ? s : 0][AFLY ? q : 0] : ra[s][q];
#pragma unroll
      for (int q = 0; q < BE; ++q)
        Bs[buf][s][bk][bn + q] = BFLY ? rb[s][q] + sgn * rbh[BFLY ? s : 0][BFLY ? q : 0] : rb[s][q];
    }
  };
  auto fetch = [&](int k0) {
    if constexpr (VEC) fetch_vec(k0);
    else fetch_one(k0);
  };
  auto stash = [&](int buf) {
    if constexpr (VEC) stash_vec(buf);
    else stash_one(buf);
  };

  acc_t acc[NS][RM][RN];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int c = 0; c < RN; ++c) acc[s][r][c] = acc_t{0, 0, 0, 0};

  // epilogue coefficients of the tile's rows and columns, staged in LDS
  // during the prologue (their load latency overlaps the first chunk's)
  constexpr bool HASEPI = EPI != EPI_NONE;
  __shared__ double Erow[HASEPI ? BM : 1], Ecol[HASEPI ? 2 : 1][HASEPI ? BN : 1];
  if constexpr (HASEPI) {
    if (tid < BM) {
      const int gm = m0 + tid;
      double v = 0.0;
      if (gm < M) v = (EPI == EPI_DIVIDE) ? ep.lz[par * H + gm] : ep.isy[gm % ep.ny] * ep.isz[gm / ep.ny];
      Erow[tid] = v;
    }
    if (tid < BN) {
      const int64_t gn = n0 + tid;
      double v0 = 0.0, v1 = 0.0;
      if (gn < NN) {
        if (EPI == EPI_DIVIDE) {
          const int g32 = (int)gn;  // position in an (nx * ny) plane: fits 32 bits
          const int bb = g32 / ep.nx, aa = g32 - bb * ep.nx;
          v0 = ep.ly[bb] + ep.lx[aa];
        } else {
          v0 = ep.isx[gn];
          v1 = ep.isx[N - 1 - gn];
        }
      }
      Ecol[0][tid] = v0;
      Ecol[HASEPI ? 1 : 0][tid] = v1;
    }
  }

  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        T af[RM], bf[RN];
#pragma unroll
        for (int r = 0; r < RM; ++r) af[r] = As[buf][s][kr][wm + 16 * r + (lane & 15)];
#pragma unroll
        for (int c = 0; c < RN; ++c) bf[c] = Bs[buf][s][kr][wn + 16 * c + (lane & 15)];
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
          for (int c = 0; c < RN; ++c)
            acc[s][r][c] = Mfma<T>::op(af[r], bf[c], acc[s][r][c]);
      }
      // inverse kinds: keep each k-step's fragment reads with its products
      // (hoisting the reads of later steps costs registers: 72 -> 56 VGPRs
      // on the 32 x 32 tiles)
      if (INV) __builtin_amdgcn_sched_barrier(0);
    }
    if (NB == 2) {
      // the other buffer was last read before the previous barrier
      if (more) stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    } else {
      __syncthreads();
      if (more) {
        stash(0);
        __syncthreads();
      }
    }
  }

#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int c = 0; c < RN; ++c) {
      const int64_t gn = n0 + wn + c * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + wm + r * 16 + Mfma<T>::row(lane, q);
        if (gm >= M || gn >= NN) continue;
        if (!INV) {
          double v = acc[0][r][c][q];
          if (RIGHT) {
            out[(int64_t)gm * N + par * H + gn] = (T)v;
          } else {
            const int mode = par * H + gm;
            if (EPI == EPI_DIVIDE) {
              const int64_t flat = (int64_t)mode * ((int64_t)ep.nx * ep.ny) + gn;
              v = (flat == ep.null3) ? 0.0
                                     : v / (Erow[wm + r * 16 + Mfma<T>::row(lane, q)] + Ecol[0][wn + c * 16 + (lane & 15)]);
            }
            out[(int64_t)mode * a.P + gn] = (T)v;
          }
        } else {
          const double t = acc[0][r][c][q], u = acc[1][r][c][q];
          double lo = t + u, hi = t - u;
          if (RIGHT) {
            const int i = (int)gn;
            if (EPI == EPI_ISQ) {
              const double syz = Erow[wm + r * 16 + Mfma<T>::row(lane, q)];
              lo *= Ecol[0][wn + c * 16 + (lane & 15)] * syz;
              hi *= Ecol[HASEPI ? 1 : 0][wn + c * 16 + (lane & 15)] * syz;
            }
            out[(int64_t)gm * N + i] = (T)lo;
            out[(int64_t)gm * N + (N - 1 - i)] = (T)hi;
          } else {
            const int i = gm;
            out[(int64_t)i * a.P + gn] = (T)lo;
            out[(int64_t)(N - 1 - i) * a.P + gn] = (T)hi;
          }
        }
      }
    }
}

// ---- bf16x3 split products (mixed form) --------------------------------------------------
// The same passes in FP32 storage, each operand split as x = hi + lo with hi
// = bf16(x) and lo = bf16(x - hi) (round to nearest even; hi + lo holds x to
// about 2^-17 relative), the product formed as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the dropped lo*lo and
// the split leave about 2^-16 relative per product).  Operands are split
// when they are stashed into LDS, where each tile is held k-contiguous
// (rows of BK bf16 plus a pad of 8), so that a lane's eight consecutive k
// values of one row or column are one 16-byte read: MFMA lane l takes
// A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i < 8, and
// holds D[4 (l / 16) + q][l % 16].  64 x 64 output tiles, four waves in a
// 2 x 2 layout, a 32-wide k chunk per LDS stage.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND, int EPI>
__global__ void __launch_bounds__(256) fd_split_bf3_kernel(SplitArgs<float> a, SplitEpi ep) {
  typedef v4f acc_t;
  constexpr int BM = 64, BN = 64, BK = 32, KP = BK + 8;
  constexpr bool INV = (KIND == RIGHT_INV || KIND == LEFT_INV);
  constexpr bool RIGHT = (KIND == RIGHT_FWD || KIND == RIGHT_INV);
  constexpr int NS = INV ? 2 : 1;
  constexpr int RM = BM / 32, RN = BN / 32;
  constexpr int AE = BM * BK / 256, BE = BK * BN / 256;
  constexpr int NB = INV ? 1 : 2;
  __shared__ __attribute__((aligned(16))) __bf16 As[NB][NS][2][BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NB][NS][2][BN][KP];

  const int pars = INV ? 1 : 2;
  const int64_t total = (int64_t)a.mtiles * a.ntiles * a.batch * pars;
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t w = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (w >= total) return;
  int mt, nt, par;
  int64_t b;
  {
    int64_t t = w;
    par = (int)(t % pars);
    t /= pars;
    if (RIGHT) {
      nt = (int)(t % a.ntiles);
      t /= a.ntiles;
      mt = (int)(t % a.mtiles);
      t /= a.mtiles;
    } else {
      mt = (int)(t % a.mtiles);
      t /= a.mtiles;
      nt = (int)(t % a.ntiles);
      t /= a.ntiles;
    }
    b = t;
  }
  if (INV) par = 0;
  const int N = a.N, H = a.H;
  const float sgn = par ? -1.0f : 1.0f;
  float* out = a.out + (RIGHT ? 0 : b * a.bstride);
  const int M = RIGHT ? (int)a.R : H;
  const int64_t NN = RIGHT ? H : a.P;
  const int K = H;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = mt * BM;
  const int64_t n0 = (int64_t)nt * BN;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  constexpr int AKT = BK / AE;                      // threads per A row (4), AE = 8 consecutive k each
  const int ar = tid / AKT, ak = (tid % AKT) * AE;
  constexpr int BNT = BN / BE;                      // threads per B row (8), BE = 8 consecutive n each
  const int bk = tid / BNT, bn = (tid % BNT) * BE;
  constexpr bool AFLY = (KIND == RIGHT_FWD), BFLY = (KIND == LEFT_FWD);
  const int64_t in_elems = RIGHT ? a.R * (int64_t)N : (int64_t)a.batch * a.bstride + (a.batch == 1 ? (int64_t)N * a.P : 0);
  const __amdgpu_buffer_rsrc_t rin = make_rsrc(a.in, in_elems);
  const __amdgpu_buffer_rsrc_t rq = make_rsrc(a.Qs, 2 * (int64_t)H * H);
  const __amdgpu_buffer_rsrc_t rqt = make_rsrc(a.QsT, 2 * (int64_t)H * H);
  const int64_t boff = RIGHT ? 0 : b * a.bstride;
  float ra[NS][AE], rb[NS][BE];
  float rah[AFLY ? NS : 1][AFLY ? AE : 1], rbh[BFLY ? NS : 1][BFLY ? BE : 1];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int ps = INV ? s : par;
#pragma unroll
      for (int q = 0; q < AE; ++q) {
        const int gm = m0 + ar, gk = k0 + ak + q;
        const bool ok = gm < M && gk < K;
        int o = OOB, oh = OOB;
        if (KIND == RIGHT_FWD) {
          o = ok ? (gm * N + gk) * 4 : OOB;
          oh = ok ? (gm * N + N - 1 - gk) * 4 : OOB;
        } else if (KIND == RIGHT_INV) {
          o = ok ? (gm * N + ps * H + gk) * 4 : OOB;
        } else {
          o = ok ? ((ps * H + gm) * H + gk) * 4 : OOB;
        }
        if (KIND == RIGHT_FWD || KIND == RIGHT_INV) ra[s][q] = bload<float>(rin, o);
        else if (KIND == LEFT_FWD) ra[s][q] = bload<float>(rqt, o);
        else ra[s][q] = bload<float>(rq, o);
        if (AFLY) rah[AFLY ? s : 0][AFLY ? q : 0] = bload<float>(rin, oh);
      }
#pragma unroll
      for (int q = 0; q < BE; ++q) {
        const int gk = k0 + bk;
        const int64_t gn = n0 + bn + q;
        const bool ok = gk < K && gn < NN;
        int o = OOB, oh = OOB;
        if (KIND == RIGHT_FWD || KIND == RIGHT_INV) {
          o = ok ? ((ps * H + gk) * H + (int)gn) * 4 : OOB;
          rb[s][q] = bload<float>(KIND == RIGHT_FWD ? rq : rqt, o);
        } else if (KIND == LEFT_FWD) {
          o = ok ? (int)((boff + (int64_t)gk * a.P + gn) * 4) : OOB;
          oh = ok ? (int)((boff + (int64_t)(N - 1 - gk) * a.P + gn) * 4) : OOB;
          rb[s][q] = bload<float>(rin, o);
          rbh[BFLY ? s : 0][BFLY ? q : 0] = bload<float>(rin, oh);
        } else {
          o = ok ? (int)((boff + (int64_t)(ps * H + gk) * a.P + gn) * 4) : OOB;
          rb[s][q] = bload<float>(rin, o);
        }
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int q = 0; q < AE; ++q) {
        const float v = AFLY ? ra[s][q] + sgn * rah[AFLY ? s : 0][AFLY ? q : 0] : ra[s][q];
        const __bf16 hi = (__bf16)v;
        As[buf][s][0][ar][ak + q] = hi;
        As[buf][s][1][ar][ak + q] = (__bf16)(v - (float)hi);
      }
#pragma unroll
      for (int q = 0; q < BE; ++q) {
        const float v = BFLY ? rb[s][q] + sgn * rbh[BFLY ? s : 0][BFLY ? q : 0] : rb[s][q];
        const __bf16 hi = (__bf16)v;
        Bs[buf][s][0][bn + q][bk] = hi;
        Bs[buf][s][1][bn + q][bk] = (__bf16)(v - (float)hi);
      }
    }
  };

  acc_t acc[NS][RM][RN];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int c = 0; c < RN; ++c) acc[s][r][c] = acc_t{0, 0, 0, 0};

  constexpr bool HASEPI = EPI != EPI_NONE;
  __shared__ double Erow[HASEPI ? BM : 1], Ecol[HASEPI ? 2 : 1][HASEPI ? BN : 1];
  if constexpr (HASEPI) {
    if (tid < BM) {
      const int gm = m0 + tid;
      double v = 0.0;
      if (gm < M) v = (EPI == EPI_DIVIDE) ? ep.lz[par * H + gm] : ep.isy[gm % ep.ny] * ep.isz[gm / ep.ny];
      Erow[tid] = v;
    }
    if (tid < BN) {
      const int64_t gn = n0 + tid;
      double v0 = 0.0, v1 = 0.0;
      if (gn < NN) {
        if (EPI == EPI_DIVIDE) {
          const int g32 = (int)gn;
          const int bb = g32 / ep.nx, aa = g32 - bb * ep.nx;
          v0 = ep.ly[bb] + ep.lx[aa];
        } else {
          v0 = ep.isx[gn];
          v1 = ep.isx[N - 1 - gn];
        }
      }
      Ecol[0][tid] = v0;
      Ecol[HASEPI ? 1 : 0][tid] = v1;
    }
  }

  const int lr = lane & 15, lk = 8 * (lane >> 4);
  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) fetch(k0 + BK);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      bf16x8 ah[RM], al[RM], bh[RN], bl[RN];
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        ah[r] = *reinterpret_cast<const bf16x8*>(&As[buf][s][0][wm + 16 * r + lr][lk]);
        al[r] = *reinterpret_cast<const bf16x8*>(&As[buf][s][1][wm + 16 * r + lr][lk]);
      }
#pragma unroll
      for (int c = 0; c < RN; ++c) {
        bh[c] = *reinterpret_cast<const bf16x8*>(&Bs[buf][s][0][wn + 16 * c + lr][lk]);
        bl[c] = *reinterpret_cast<const bf16x8*>(&Bs[buf][s][1][wn + 16 * c + lr][lk]);
      }
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int c = 0; c < RN; ++c) {
          acc[s][r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[r], bh[c], acc[s][r][c], 0, 0, 0);
          acc[s][r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bl[c], acc[s][r][c], 0, 0, 0);
          acc[s][r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bh[c], acc[s][r][c], 0, 0, 0);
        }
    }
    if (NB == 2) {
      if (more) stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    } else {
      __syncthreads();
      if (more) {
        stash(0);
        __syncthreads();
      }
    }
  }

#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int c = 0; c < RN; ++c) {
      const int64_t gn = n0 + wn + c * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int lrow = wm + r * 16 + 4 * (lane >> 4) + q;
        const int gm = m0 + lrow;
        if (gm >= M || gn >= NN) continue;
        if (!INV) {
          double v = acc[0][r][c][q];
          if (RIGHT) {
            out[(int64_t)gm * N + par * H + gn] = (float)v;
          } else {
            const int mode = par * H + gm;
            if (EPI == EPI_DIVIDE) {
              const int64_t flat = (int64_t)mode * ((int64_t)ep.nx * ep.ny) + gn;
              v = (flat == ep.null3) ? 0.0 : v / (Erow[lrow] + Ecol[0][wn + c * 16 + (lane & 15)]);
            }
            out[(int64_t)mode * a.P + gn] = (float)v;
          }
        } else {
          const double t = acc[0][r][c][q], u = acc[1][r][c][q];
          double lo = t + u, hi = t - u;
          if (RIGHT) {
            const int i = (int)gn;
            if (EPI == EPI_ISQ) {
              const double syz = Erow[lrow];
              lo *= Ecol[0][wn + c * 16 + (lane & 15)] * syz;
              hi *= Ecol[HASEPI ? 1 : 0][wn + c * 16 + (lane & 15)] * syz;
            }
            out[(int64_t)gm * N + i] = (float)lo;
            out[(int64_t)gm * N + (N - 1 - i)] = (float)hi;
          } else {
            const int i = gm;
            out[(int64_t)i * a.P + gn] = (float)lo;
            out[(int64_t)(N - 1 - i) * a.P + gn] = (float)hi;
          }
        }
      }
    }
}

template <int KIND, int EPI>
hipError_t launch_bf3(const SplitArgs<float>& a0, const SplitEpi& ep, hipStream_t s) {
  SplitArgs<float> a = a0;
  const bool inv = (KIND == RIGHT_INV || KIND == LEFT_INV);
  const bool right = (KIND == RIGHT_FWD || KIND == RIGHT_INV);
  const int64_t M = right ? a.R : a.H;
  const int64_t NN = right ? a.H : a.P;
  a.mtiles = (int)((M + 63) / 64);
  a.ntiles = (int)((NN + 63) / 64);
  const int64_t total = (int64_t)a.mtiles * a.ntiles * a.batch * (inv ? 1 : 2);
  const int64_t blocks = ((total + 7) / 8) * 8;
  fd_split_bf3_kernel<KIND, EPI><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, ep);
  return hipGetLastError();
}

hipError_t split_pass_bf3(const kv_ctx* c, int axis, bool inverse, int epi, const float* in, float* out) {
  const Grid& g = c->g;
  SplitArgs<float> a{};
  a.in = in;
  a.out = out;
  a.Qs = c->Qf32[axis];
  a.QsT = c->Qt32[axis];
  a.N = g.ax[axis].n;
  a.H = a.N / 2;
  a.batch = 1;
  const int64_t nx = g.nx, ny = g.ny, nz = g.nz;
  if (axis == 0) {
    a.R = ny * nz;
  } else if (axis == 1) {
    a.P = nx;
    a.bstride = nx * ny;
    a.batch = (int)nz;
  } else {
    a.P = nx * ny;
  }
  SplitEpi ep{g.ax[0].lam, g.ax[1].lam, g.ax[2].lam, g.ax[0].isq, g.ax[1].isq, g.ax[2].isq,
              g.nx, g.ny, g.null3};
  hipStream_t s = c->stream;
  if (axis == 0) {
    if (!inverse) return launch_bf3<RIGHT_FWD, EPI_NONE>(a, ep, s);
    if (epi == 2) return launch_bf3<RIGHT_INV, EPI_ISQ>(a, ep, s);
    return launch_bf3<RIGHT_INV, EPI_NONE>(a, ep, s);
  }
  if (!inverse) {
    if (epi == 1) return launch_bf3<LEFT_FWD, EPI_DIVIDE>(a, ep, s);
    return launch_bf3<LEFT_FWD, EPI_NONE>(a, ep, s);
  }
  return launch_bf3<LEFT_INV, EPI_NONE>(a, ep, s);
}

// Pair loads on by default; KV_FD_PAIRS=0 selects one element per load
// (read at every launch, so tests can cover both paths in one process).
bool pair_loads() {
  const char* e = getenv("KV_FD_PAIRS");
  return !(e && atoi(e) == 0);
}

template <typename T, int KIND, int EPI, int BM, int BN, int BK>
hipError_t launch_tiles(const SplitArgs<T>& a0, const SplitEpi& ep, hipStream_t s) {
  SplitArgs<T> a = a0;
  const bool inv = (KIND == RIGHT_INV || KIND == LEFT_INV);
  const bool right = (KIND == RIGHT_FWD || KIND == RIGHT_INV);
  const int64_t M = right ? a.R : a.H;
  const int64_t NN = right ? a.H : a.P;
  a.mtiles = (int)((M + BM - 1) / BM);
  a.ntiles = (int)((NN + BN - 1) / BN);
  const int64_t total = (int64_t)a.mtiles * a.ntiles * a.batch * (inv ? 1 : 2);
  const int64_t blocks = ((total + 7) / 8) * 8;
  // pairs stay inside a row and aligned when the half size and the line
  // length are even
  const bool vec = (a.H % 2 == 0) && (right || a.P % 2 == 0) && pair_loads();
  if (vec)
    fd_split_kernel<T, KIND, EPI, BM, BN, BK, true><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, ep);
  else
    fd_split_kernel<T, KIND, EPI, BM, BN, BK, false><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, ep);
  return hipGetLastError();
}

// Tile shapes (FP64, measured at H = 128): the forward kinds without an
// epilogue take 128 x 128 tiles once the half size fills them (four times the
// MFMA work per prologue and epilogue of a 64 x 64 tile); the spectral-divide
// kind keeps 64 x 64 (at 128 x 128 it fits two waves per SIMD, but the whole
// projection measured 5 us slower); the inverse kinds keep 64 x 64, because
// their two accumulator sets double the registers per output.  Small grids take 32 x 32 tiles when 64 x 64 ones
// would leave fewer than about four blocks per CU.  FP32 (mixed form) follows
// the same rules without the 128 x 128 case.  KV_FD_TILE=64 or 32 forces one
// shape (fd_forced_tile, read at every launch, for tests and measurements).
template <typename T, int KIND, int EPI>
hipError_t launch(const SplitArgs<T>& a, const SplitEpi& ep, hipStream_t s) {
  const bool inv = (KIND == RIGHT_INV || KIND == LEFT_INV);
  const bool right = (KIND == RIGHT_FWD || KIND == RIGHT_INV);
  const int forced = fd_forced_tile();
  if (forced == 64) return launch_tiles<T, KIND, EPI, 64, 64, 16>(a, ep, s);
  if (forced == 32) return launch_tiles<T, KIND, EPI, 32, 32, 16>(a, ep, s);
  if constexpr (sizeof(T) == 8 && KIND != RIGHT_INV && KIND != LEFT_INV && EPI == EPI_NONE) {
    if (a.H >= 128) return launch_tiles<T, KIND, EPI, 128, 128, 16>(a, ep, s);
  }
  const int64_t M = right ? a.R : a.H, NN = right ? a.H : a.P;
  const int64_t tiles64 = ((M + 63) / 64) * ((NN + 63) / 64) * a.batch * (inv ? 1 : 2);
  if (tiles64 < 1024) return launch_tiles<T, KIND, EPI, 32, 32, 16>(a, ep, s);
  return launch_tiles<T, KIND, EPI, 64, 64, 16>(a, ep, s);
}

template <typename T>
hipError_t split_pass(const kv_ctx* c, int axis, bool inverse, int epi, const T* in, T* out, const T* Qs,
                      const T* QsT) {
  const Grid& g = c->g;
  SplitArgs<T> a{};
  a.in = in;
  a.out = out;
  a.Qs = Qs;
  a.QsT = QsT;
  a.N = g.ax[axis].n;
  a.H = a.N / 2;
  a.batch = 1;
  const int64_t nx = g.nx, ny = g.ny, nz = g.nz;
  if (axis == 0) {
    a.R = ny * nz;
  } else if (axis == 1) {
    a.P = nx;
    a.bstride = nx * ny;
    a.batch = (int)nz;
  } else {
    a.P = nx * ny;
  }
  SplitEpi ep{g.ax[0].lam, g.ax[1].lam, g.ax[2].lam, g.ax[0].isq, g.ax[1].isq, g.ax[2].isq,
              g.nx, g.ny, g.null3};
  hipStream_t s = c->stream;
  if (axis == 0) {
    if (!inverse) return launch<T, RIGHT_FWD, EPI_NONE>(a, ep, s);
    if (epi == 2) return launch<T, RIGHT_INV, EPI_ISQ>(a, ep, s);
    return launch<T, RIGHT_INV, EPI_NONE>(a, ep, s);
  }
  if (!inverse) {
    if (epi == 1) return launch<T, LEFT_FWD, EPI_DIVIDE>(a, ep, s);
    return launch<T, LEFT_FWD, EPI_NONE>(a, ep, s);
  }
  return launch<T, LEFT_INV, EPI_NONE>(a, ep, s);
}

}  // namespace

int fd_forced_tile() {
  const char* e = getenv("KV_FD_TILE");
  if (!e) return 0;
  const int t = atoi(e);
  return (t == 64 || t == 32) ? t : 0;
}

// One axis pass of the split transform.  axis 0 (x): RIGHT kinds on rows of
// length nx; axis 1 (y): LEFT kinds on lines of nx, batched over z; axis 2
// (z): LEFT kinds on lines of nx*ny.  epi: 0 none, 1 spectral divide (z
// forward), 2 S^-1 scaling (x inverse).
hipError_t launch_fd_split_pass(const kv_ctx* c, int axis, bool inverse, int epi, const double* in, double* out) {
  return split_pass<double>(c, axis, inverse, epi, in, out, c->Qf[axis], c->Qt[axis]);
}

// The same in FP32 storage on the FP32 matrix cores (mixed form).
hipError_t launch_fd_split_pass_f32(const kv_ctx* c, int axis, bool inverse, int epi, const float* in, float* out) {
  return split_pass<float>(c, axis, inverse, epi, in, out, c->Qf32[axis], c->Qt32[axis]);
}

// The six passes with bf16x3 split products (FP32 storage): in (scaled
// divergence) -> out (pressure); every axis must be split.  in is overwritten.
hipError_t launch_fd_solve_bf3(const kv_ctx* c, float* in, float* out) {
  float* A = in;
  float* Bf = reinterpret_cast<float*>(c->cellB);
  hipError_t e;
  if ((e = split_pass_bf3(c, 0, false, 0, A, Bf))) return e;
  if ((e = split_pass_bf3(c, 1, false, 0, Bf, A))) return e;
  if ((e = split_pass_bf3(c, 2, false, 1, A, Bf))) return e;
  if ((e = split_pass_bf3(c, 2, true, 0, Bf, A))) return e;
  if ((e = split_pass_bf3(c, 1, true, 0, A, Bf))) return e;
  return split_pass_bf3(c, 0, true, 2, Bf, out);
}

// Poisson solve in FP32 storage: in (scaled divergence) -> out (pressure);
// every axis must be split.  in is overwritten.
hipError_t launch_fd_solve_f32(const kv_ctx* c, float* in, float* out) {
  float* A = in;
  float* Bf = reinterpret_cast<float*>(c->cellB);
  hipError_t e;
  if ((e = launch_fd_split_pass_f32(c, 0, false, 0, A, Bf))) return e;
  if ((e = launch_fd_split_pass_f32(c, 1, false, 0, Bf, A))) return e;
  if ((e = launch_fd_split_pass_f32(c, 2, false, 1, A, Bf))) return e;
  if ((e = launch_fd_split_pass_f32(c, 2, true, 0, Bf, A))) return e;
  if ((e = launch_fd_split_pass_f32(c, 1, true, 0, A, Bf))) return e;
  return launch_fd_split_pass_f32(c, 0, true, 2, Bf, out);
}

}  // namespace kv
