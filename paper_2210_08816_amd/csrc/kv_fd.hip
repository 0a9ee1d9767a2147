// Pressure Poisson solve L p = r, L = D G, by fast diagonalization.
//
// L = sum_a H_a^-1 K_a with K_a symmetric tridiagonal (Neumann), so with
// S = (H_x H_y H_z)^1/2 and M_a = H_a^-1/2 K_a H_a^-1/2 = Q_a Lam_a Q_a^T,
//   p = S^-1 (Q_x Q_y Q_z) (Lam_x + Lam_y + Lam_z)^+ (Q_x Q_y Q_z)^T S r.
// Each 1-D transform is a dense GEMM along one axis of the (z, y, x) cell
// field, done on the FP64 matrix cores (v_mfma_f64_16x16x4):
//   x: C (ny nz x nx) = F (ny nz x nx) * Q_x            (rows contiguous)
//   y: C_k (ny x nx)  = Q_y^T * F_k (ny x nx), k < nz    (batched)
//   z: C (nz x nx ny) = Q_z^T * F (nz x nx ny)
// None needs a transpose in memory.  The spectral divide is fused into the
// epilogue of the last forward pass, the S^-1 scaling into the last inverse
// pass; the S r scaling is fused into the divergence kernel that produces r.
#include "kv_internal.h"

namespace kv {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

enum { EPI_NONE = 0, EPI_DIVIDE = 1, EPI_ISQ = 2 };

struct Epi {
  const double *lx, *ly, *lz;     // per-axis eigenvalues
  const double *isx, *isy, *isz;  // 1/sqrt(h) per axis
  int nx, ny;
  int64_t null3;                  // flat (c, b, a) index of the constant mode (-1: none)
  double sigma, coef;             // divide by sigma + coef (lx + ly + lz)
};

constexpr int BK = 16;

// One batched product C[b] = A[b] * B[b] (row-major) of a launch.
struct GemmProb {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, sA, ldb, sB, ldc, sC;
  int M, N, K, mtiles, ntiles, batch, a_is_big;
  int64_t first;  // first work item of this product in the launch
  Epi ep;
};
constexpr int MAXP = 4;
struct GemmSet {
  GemmProb p[MAXP];
  int np;
  int64_t total;  // work items (64x64 output tiles) over all products
};

// Up to four independent products (the four blocks of a packed vector) in
// one launch, 256 threads = 4 waves, TILE x TILE output tile per block (64,
// or 32 on small grids), each wave a quarter as (TILE/32)^2 MFMA 16x16
// accumulators.  Within a product, work items are
// laid out so that the blocks sharing the large operand's tile are
// consecutive on one XCD (blocks are dealt round-robin over the 8 XCDs).
template <int EPI, int TILE>
__global__ void __launch_bounds__(256) fd_gemm_kernel(GemmSet gs) {
  constexpr int BM = TILE, BN = TILE, R = TILE / 32;  // R x R accumulators per wave
  constexpr int AE = BM * BK / 256, BE = BK * BN / 256;  // tile elements per thread
  __shared__ double As[BK][BM + 2];  // [k][m]
  __shared__ double Bs[BK][BN + 2];  // [k][n]
  const int64_t per_xcd = (gs.total + 7) / 8;
  const int64_t f = blockIdx.x;
  int64_t w = (f % 8) * per_xcd + f / 8;
  if (w >= gs.total) return;
  int q = 0;
#pragma unroll
  for (int t = 1; t < MAXP; ++t)
    if (t < gs.np && w >= gs.p[t].first) q = t;
  GemmProb P;
  switch (q) {  // constant indices: the fields stay scalar kernel-argument loads
    case 0: P = gs.p[0]; break;
    case 1: P = gs.p[1]; break;
    case 2: P = gs.p[2]; break;
    default: P = gs.p[3]; break;
  }
  w -= P.first;
  const int M = P.M, N = P.N, K = P.K, mtiles = P.mtiles, ntiles = P.ntiles;
  const int64_t lda = P.lda, ldb = P.ldb, ldc = P.ldc;
  const Epi& ep = P.ep;
  int mt, nt;
  int64_t b;
  if (P.a_is_big) {  // A tile shared by the ntiles blocks of one row of tiles
    nt = (int)(w % ntiles);
    mt = (int)((w / ntiles) % mtiles);
    b = w / ((int64_t)ntiles * mtiles);
  } else {           // B tile shared by the mtiles blocks of one column of tiles
    mt = (int)(w % mtiles);
    nt = (int)((w / mtiles) % ntiles);
    b = w / ((int64_t)ntiles * mtiles);
  }
  const double* __restrict__ A = P.A + b * P.sA;
  const double* __restrict__ B = P.B + b * P.sB;
  double* __restrict__ C = P.C + b * P.sC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = mt * BM, n0 = nt * BN;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  v4d acc[R][R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < R; ++c) acc[r][c] = v4d{0, 0, 0, 0};

  const int ar = tid / (BK / AE), ak = (tid % (BK / AE)) * AE;  // A tile: row, first k
  const int bk = tid / (BN / BE), bn = (tid % (BN / BE)) * BE;  // B tile: k, first n
  for (int k0 = 0; k0 < K; k0 += BK) {
    {
      const int gm = m0 + ar;
#pragma unroll
      for (int q = 0; q < AE; ++q) {
        const int gk = k0 + ak + q;
        As[ak + q][ar] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : 0.0;
      }
    }
    {
      const int gk = k0 + bk;
#pragma unroll
      for (int q = 0; q < BE; ++q) {
        const int gn = n0 + bn + q;
        Bs[bk][bn + q] = (gk < K && gn < N) ? B[(int64_t)gk * ldb + gn] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double af[R], bf[R];
#pragma unroll
      for (int r = 0; r < R; ++r) af[r] = As[kr][wm + 16 * r + (lane & 15)];
#pragma unroll
      for (int c = 0; c < R; ++c) bf[c] = Bs[kr][wn + 16 * c + (lane & 15)];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[r], bf[c], acc[r][c], 0, 0, 0);
    }
    __syncthreads();
  }

  // D[i][j] of a 16x16 block: lane = j + 16 * (i % 4), element i / 4.
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int cblk = 0; cblk < R; ++cblk) {
      const int gn = n0 + wn + cblk * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + wm + r * 16 + (lane >> 4) + 4 * q;
        if (gm < M && gn < N) {
          double v = acc[r][cblk][q];
          if (EPI == EPI_DIVIDE) {
            // C is (nz x nx*ny): m = z-mode c, n = b * nx + a
            const int bb = gn / ep.nx, a = gn - bb * ep.nx;
            const int64_t flat = (int64_t)gm * ((int64_t)ep.nx * ep.ny) + gn;
            const double den = ep.sigma + ep.coef * (ep.lz[gm] + ep.ly[bb] + ep.lx[a]);
            v = (flat == ep.null3) ? 0.0 : v / den;
          } else if (EPI == EPI_ISQ) {
            // C is (ny*nz x nx): m = k * ny + j, n = i
            const int j = gm % ep.ny, k = gm / ep.ny;
            v *= ep.isx[gn] * ep.isy[j] * ep.isz[k];
          }
          C[(int64_t)gm * ldc + gn] = v;
        }
      }
    }
}

GemmProb prob(const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double* C,
              int64_t ldc, int64_t sC, int M, int N, int K, int batch, int a_is_big, const Epi& ep) {
  GemmProb p{};
  p.A = A;
  p.B = B;
  p.C = C;
  p.lda = lda;
  p.sA = sA;
  p.ldb = ldb;
  p.sB = sB;
  p.ldc = ldc;
  p.sC = sC;
  p.M = M;
  p.N = N;
  p.K = K;
  p.batch = batch;
  p.a_is_big = a_is_big;
  p.ep = ep;
  return p;
}

// Tiles of 64 x 64, or 32 x 32 when 64 x 64 ones would give fewer than about
// four blocks per CU (KV_FD_TILE forces either).
template <int EPI>
hipError_t gemm_set(const GemmProb* ps, int np, hipStream_t s) {
  int64_t tiles64 = 0;
  for (int q = 0; q < np; ++q) tiles64 += (int64_t)((ps[q].M + 63) / 64) * ((ps[q].N + 63) / 64) * ps[q].batch;
  const int forced = fd_forced_tile();
  const int tile = forced ? forced : (tiles64 < 1024 ? 32 : 64);
  GemmSet gs{};
  gs.np = np;
  int64_t total = 0;
  for (int q = 0; q < np; ++q) {
    gs.p[q] = ps[q];
    gs.p[q].mtiles = (ps[q].M + tile - 1) / tile;
    gs.p[q].ntiles = (ps[q].N + tile - 1) / tile;
    gs.p[q].first = total;
    total += (int64_t)gs.p[q].mtiles * gs.p[q].ntiles * ps[q].batch;
  }
  gs.total = total;
  if (total == 0) return hipSuccess;
  const int64_t blocks = ((total + 7) / 8) * 8;
  if (tile == 32)
    fd_gemm_kernel<EPI, 32><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(gs);
  else
    fd_gemm_kernel<EPI, 64><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(gs);
  return hipGetLastError();
}

template <int EPI>
hipError_t gemm(const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
                double* C, int64_t ldc, int64_t sC, int M, int N, int K, int batch, int a_is_big,
                const Epi& ep, hipStream_t s) {
  const GemmProb p = prob(A, lda, sA, B, ldb, sB, C, ldc, sC, M, N, K, batch, a_is_big, ep);
  return gemm_set<EPI>(&p, 1, s);
}

}  // namespace

hipError_t launch_fd_solve(const kv_ctx* c, double* in, double* out) {
  const Grid& g = c->g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t plane = (int64_t)nx * ny;
  Epi ep{g.ax[0].lam, g.ax[1].lam, g.ax[2].lam, g.ax[0].isq, g.ax[1].isq, g.ax[2].isq, nx, ny, g.null3, 0.0, 1.0};
  double* A = in;
  double* Bf = c->cellB;
  hipStream_t s = c->stream;
  hipError_t e;
  // forward: x, y, z (+ divide); mirror-symmetric axes use the half-size split
  if (c->split[0]) e = launch_fd_split_pass(c, 0, false, 0, A, Bf);
  else e = gemm<EPI_NONE>(A, nx, 0, c->Qf[0], nx, 0, Bf, nx, 0, ny * nz, nx, nx, 1, 1, ep, s);
  if (e) return e;
  if (c->split[1]) e = launch_fd_split_pass(c, 1, false, 0, Bf, A);
  else e = gemm<EPI_NONE>(c->Qt[1], ny, 0, Bf, nx, plane, A, nx, plane, ny, nx, ny, nz, 0, ep, s);
  if (e) return e;
  if (c->split[2]) e = launch_fd_split_pass(c, 2, false, 1, A, Bf);
  else e = gemm<EPI_DIVIDE>(c->Qt[2], nz, 0, A, plane, 0, Bf, plane, 0, nz, (int)plane, nz, 1, 0, ep, s);
  if (e) return e;
  // inverse: z, y, x (+ S^-1)
  if (c->split[2]) e = launch_fd_split_pass(c, 2, true, 0, Bf, A);
  else e = gemm<EPI_NONE>(c->Qf[2], nz, 0, Bf, plane, 0, A, plane, 0, nz, (int)plane, nz, 1, 0, ep, s);
  if (e) return e;
  if (c->split[1]) e = launch_fd_split_pass(c, 1, true, 0, A, Bf);
  else e = gemm<EPI_NONE>(c->Qf[1], ny, 0, A, nx, plane, Bf, nx, plane, ny, nx, ny, nz, 0, ep, s);
  if (e) return e;
  if (c->split[0]) return launch_fd_split_pass(c, 0, true, 2, Bf, out);
  return gemm<EPI_ISQ>(Bf, nx, 0, c->Qt[0], nx, 0, out, nx, 0, ny * nz, nx, nx, 1, 1, ep, s);
}

// The four Helmholtz solves of a packed vector (one per block u, v, w, T,
// each on its own grid and bases), pass by pass: each of the six passes is
// one launch over the four products.  The passes alternate between out and
// scr (in is read by the first pass only, so in == out is allowed).
hipError_t launch_fd_helmholtz4(const kv_ctx* c, const HelmBasis* const bx[4], const HelmBasis* const by[4],
                                const HelmBasis* const bz[4], double sigma, const double coef[4],
                                const double* const in[4], double* const out[4], double* const scr[4]) {
  hipStream_t s = c->stream;
  GemmProb ps[4];
  hipError_t e;
  // forward x, y, z (+ divide), inverse z, y, x; the H^1/2 scalings sit in the bases
  for (int pass = 0; pass < 6; ++pass) {
    for (int q = 0; q < 4; ++q) {
      const HelmBasis &X = *bx[q], &Y = *by[q], &Z = *bz[q];
      const int nx = X.n, ny = Y.n, nz = Z.n;
      const int64_t plane = (int64_t)nx * ny;
      const Epi ep{X.lam, Y.lam, Z.lam, nullptr, nullptr, nullptr, nx, ny, -1, sigma, coef[q]};
      const double* src = pass == 0 ? in[q] : (pass % 2 ? scr[q] : out[q]);
      double* dst = pass % 2 ? out[q] : scr[q];
      switch (pass) {
        case 0: ps[q] = prob(src, nx, 0, X.fwdB, nx, 0, dst, nx, 0, ny * nz, nx, nx, 1, 1, ep); break;
        case 1: ps[q] = prob(Y.fwdA, ny, 0, src, nx, plane, dst, nx, plane, ny, nx, ny, nz, 0, ep); break;
        case 2: ps[q] = prob(Z.fwdA, nz, 0, src, plane, 0, dst, plane, 0, nz, (int)plane, nz, 1, 0, ep); break;
        case 3: ps[q] = prob(Z.invA, nz, 0, src, plane, 0, dst, plane, 0, nz, (int)plane, nz, 1, 0, ep); break;
        case 4: ps[q] = prob(Y.invA, ny, 0, src, nx, plane, dst, nx, plane, ny, nx, ny, nz, 0, ep); break;
        default: ps[q] = prob(src, nx, 0, X.invB, nx, 0, dst, nx, 0, ny * nz, nx, nx, 1, 1, ep); break;
      }
    }
    e = pass == 2 ? gemm_set<EPI_DIVIDE>(ps, 4, s) : gemm_set<EPI_NONE>(ps, 4, s);
    if (e) return e;
  }
  return hipSuccess;
}

}  // namespace kv
