// Eigenvalues and selected eigenvectors of the small upper-Hessenberg matrix
// H_m that Arnoldi builds (Ritz values and Ritz coefficient vectors of the
// Chebyshev-preconditioned Arnoldi method, paper Sec. 1 and Sec. 3).
//
// One wavefront does all of it, FP64:
//   1. Francis implicit double-shift QR on the active window (eigenvalues
//      only), deflating when |h_{l,l-1}| <= eps (|h_{l-1,l-1}| + |h_{l,l}|);
//      ad-hoc shifts after every 10 iterations without deflation.  Each
//      3x3 reflector is formed redundantly by every lane and applied to the
//      rows / columns with one matrix element per lane.
//   2. For each requested eigenvalue, inverse iteration on H - lambda I in
//      complex arithmetic: Hessenberg LU with partial pivoting between
//      adjacent rows, two solves, unit 2-norm result.
// H and the work matrices live in a device scratch buffer (small, cached).
#include "kv_internal.h"

namespace kv {
namespace {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // scaled division (Smith)
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + r * b.im;
    return {(a.re + r * a.im) / d, (a.im - r * a.re) / d};
  }
  const double r = b.re / b.im, d = b.im + r * b.re;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

// Francis double-shift QR; H row-major m x m with leading dimension m, destroyed.
__global__ void __launch_bounds__(64) hqr_kernel(double* __restrict__ H, int m, double* __restrict__ wr,
                                                 double* __restrict__ wi, int* __restrict__ info) {
  const int lane = threadIdx.x;
  const double eps = 2.220446049250313e-16;
  auto h = [&](int r, int c) -> double& { return H[(int64_t)r * m + c]; };
  double anorm = 0.0;
  for (int r = 0; r < m; ++r)
    for (int c = (r > 0 ? r - 1 : 0); c < m; ++c) anorm += fabs(h(r, c));
  int hi = m - 1, its = 0, total = 0;
  int status = 0;
  while (hi >= 0) {
    // find the start l of the unreduced active block ending at hi
    // (after 100 iterations without a deflation the test relaxes to
    // sqrt(eps): a nearly defective cluster, whose subdiagonal decays only
    // linearly, is taken as converged; its values carry the cluster's own
    // ill-conditioning, eps^(1/p) for p coalescing values)
    const double tol = its < 100 ? eps : 1.4901161193847656e-08;
    // the largest l <= hi with a negligible h(l, l-1) (0 if none), 64
    // candidates per round, one per lane (lane 0 the highest): the reads of a
    // round are independent instead of one dependent read per candidate
    int l = 0;
    for (int top = hi; top > 0; top -= 64) {
      const int cand = top - lane;
      bool neg = false, strict = false;
      if (cand > 0) {
        double sc = fabs(h(cand - 1, cand - 1)) + fabs(h(cand, cand));
        if (sc == 0.0) sc = anorm;
        const double sub = fabs(h(cand, cand - 1));
        neg = sub <= tol * sc;
        strict = sub <= eps * sc;
      }
      const unsigned long long hit = __ballot(neg);
      if (hit) {
        const int first = __ffsll((long long)hit) - 1;
        l = top - first;
        if (!((__ballot(strict) >> first) & 1ull)) status |= 2;  // deflated by the relaxed test only
        break;
      }
    }
    if (l == hi) {
      if (lane == 0) {
        wr[hi] = h(hi, hi);
        wi[hi] = 0.0;
      }
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      const double a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
      const double p = 0.5 * (a - d), q = p * p + b * c;
      if (lane == 0) {
        if (q >= 0.0) {
          const double zz = p + copysign(sqrt(q), p);
          const double l1 = d + zz;
          const double l2 = (zz != 0.0) ? d - b * c / zz : d + zz;
          wr[hi - 1] = l1;
          wr[hi] = l2;
          wi[hi - 1] = wi[hi] = 0.0;
        } else {
          const double im = sqrt(-q);
          wr[hi - 1] = wr[hi] = d + p;
          wi[hi - 1] = im;
          wi[hi] = -im;
        }
      }
      hi -= 2;
      its = 0;
      continue;
    }
    // iteration limits as LAPACK's small-bulge QR: 30 max(10, m) per
    // deflation, and a bound on the total
    const int lim = 30 * (m > 10 ? m : 10);
    if (its > lim || total > 4 * lim) {
      status |= 1;
      break;
    }
    ++its;
    ++total;
    // double shift (sum s, product t) from a 2x2: the trailing one, or every
    // tenth iteration without a deflation an exceptional pair
    // [g + 0.75e, -0.4375e; e, g + 0.75e] centred at the bottom (tenth) or top
    // (twentieth) diagonal entry of the block, as in LAPACK's small-bulge QR.
    // Complex eigenvalues of the 2x2 give a conjugate pair; real ones give
    // the one nearer its last diagonal entry twice.
    double h11, h12, h21, h22;
    if (its % 20 == 0) {
      const double e = fabs(h(l + 1, l)) + fabs(h(l + 2, l + 1));
      h11 = h22 = h(l, l) + 0.75 * e;
      h12 = -0.4375 * e;
      h21 = e;
    } else if (its % 10 == 0) {
      const double e = fabs(h(hi, hi - 1)) + fabs(h(hi - 1, hi - 2));
      h11 = h22 = h(hi, hi) + 0.75 * e;
      h12 = -0.4375 * e;
      h21 = e;
    } else {
      h11 = h(hi - 1, hi - 1);
      h12 = h(hi - 1, hi);
      h21 = h(hi, hi - 1);
      h22 = h(hi, hi);
    }
    double s = 0.0, t = 0.0;
    const double sc = fabs(h11) + fabs(h12) + fabs(h21) + fabs(h22);
    if (sc != 0.0) {
      h11 /= sc;
      h12 /= sc;
      h21 /= sc;
      h22 /= sc;
      const double tr = 0.5 * (h11 + h22);
      const double det = (h11 - tr) * (h22 - tr) - h12 * h21;
      const double rtd = sqrt(fabs(det));
      if (det >= 0.0) {
        s = 2.0 * tr * sc;
        t = (tr * sc) * (tr * sc) + (rtd * sc) * (rtd * sc);
      } else {
        const double r1 = tr + rtd, r2 = tr - rtd;
        const double rr = (fabs(r1 - h22) <= fabs(r2 - h22) ? r1 : r2) * sc;
        s = 2.0 * rr;
        t = rr * rr;
      }
    }
    // first column of (H - s1 I)(H - s2 I) restricted to the block
    double x = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t;
    double y = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s);
    double z = h(l + 1, l) * h(l + 2, l + 1);
    for (int k = l - 1; k <= hi - 2; ++k) {
      const int nr = (k < hi - 2) ? 3 : 2;  // reflector size
      // Householder v with (I - tau v v^T)(x,y,z)^T = (beta,0,0)^T, v0 = 1
      // (no barrier here: x, y, z are in registers before any store below
      // can be issued, and the entries the row update reads were ordered by
      // the previous step's second barrier)
      const double nrm = sqrt(x * x + y * y + (nr == 3 ? z * z : 0.0));
      if (nrm != 0.0) {
        const double beta = (x >= 0.0) ? -nrm : nrm;
        const double v0 = x - beta;
        const double iv0 = 1.0 / v0;
        const double v1 = y * iv0, v2 = (nr == 3) ? z * iv0 : 0.0;
        const double tau = (beta - x) / beta;
        const int r0 = k + 1;
        // rows r0..r0+nr-1, columns max(k, l)..hi
        const int cs = (k > l ? k : l);
        for (int c = cs + lane; c <= hi; c += 64) {
          double a0 = h(r0, c), a1 = h(r0 + 1, c), a2 = (nr == 3) ? h(r0 + 2, c) : 0.0;
          const double dd = tau * (a0 + v1 * a1 + v2 * a2);
          h(r0, c) = a0 - dd;
          h(r0 + 1, c) = a1 - dd * v1;
          if (nr == 3) h(r0 + 2, c) = a2 - dd * v2;
        }
        __syncthreads();
        // columns r0..r0+nr-1, rows l..min(k+4, hi)
        const int re = (k + 4 < hi) ? k + 4 : hi;
        for (int r = l + lane; r <= re; r += 64) {
          double a0 = h(r, r0), a1 = h(r, r0 + 1), a2 = (nr == 3) ? h(r, r0 + 2) : 0.0;
          const double dd = tau * (a0 + v1 * a1 + v2 * a2);
          h(r, r0) = a0 - dd;
          h(r, r0 + 1) = a1 - dd * v1;
          if (nr == 3) h(r, r0 + 2) = a2 - dd * v2;
        }
        __syncthreads();
        if (k >= l) {
          // the bulge column below the subdiagonal is now zero (column k is
          // not read again in this sweep: no barrier)
          if (lane == 0) {
            h(k + 2, k) = 0.0;
            if (nr == 3) h(k + 3, k) = 0.0;
          }
        }
      }
      if (k + 1 <= hi - 2) {
        x = h(k + 2, k + 1);
        y = h(k + 3, k + 1);
        z = (k + 1 < hi - 2) ? h(k + 4, k + 1) : 0.0;
      }
    }
  }
  if (lane == 0) info[0] = status;
}

// Inverse iteration for eigenvalue (lr, li) of the original H (row-major m x m):
// W is complex scratch m*m, b complex scratch m; result unit 2-norm in (vr, vi).
__global__ void __launch_bounds__(64) inviter_kernel(const double* __restrict__ H, int m, const double* __restrict__ lr,
                                                     const double* __restrict__ li, int nsel,
                                                     cplx* __restrict__ Wall, cplx* __restrict__ ball,
                                                     double* __restrict__ vr, double* __restrict__ vi) {
  const int lane = threadIdx.x;
  const int q = blockIdx.x;
  if (q >= nsel) return;
  cplx* W = Wall + (int64_t)q * m * m;
  cplx* b = ball + (int64_t)q * m;
  __shared__ int piv[512];
  const cplx lam = {lr[q], li[q]};
  // max |H| over the matrix: a strided maximum per lane, then across the
  // wave (a maximum is exact in any order)
  double hn = 0.0;
  for (int e = lane; e < m * m; e += 64) hn = fmax(hn, fabs(H[e]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) hn = fmax(hn, __shfl_xor(hn, o, 64));
  const double tiny = 1e-15 * (hn > 0.0 ? hn : 1.0);
  // W = H - lambda I
  for (int e = lane; e < m * m; e += 64) {
    const int r = e / m, c = e % m;
    W[e] = {H[e] - (r == c ? lam.re : 0.0), (r == c ? -lam.im : 0.0)};
  }
  for (int r = lane; r < m; r += 64) b[r] = {1.0, 0.0};
  __syncthreads();
  // LU with partial pivoting between rows k and k+1 (Hessenberg)
  for (int k = 0; k < m - 1; ++k) {
    const cplx p = W[(int64_t)k * m + k], sub = W[(int64_t)(k + 1) * m + k];
    const bool sw = cabs2(sub) > cabs2(p);
    __syncthreads();
    if (sw)
      for (int c = k + lane; c < m; c += 64) {
        const cplx t = W[(int64_t)k * m + c];
        W[(int64_t)k * m + c] = W[(int64_t)(k + 1) * m + c];
        W[(int64_t)(k + 1) * m + c] = t;
      }
    if (lane == 0) piv[k] = sw ? 1 : 0;
    __syncthreads();
    cplx d = W[(int64_t)k * m + k];
    if (cabs2(d) == 0.0) d = {tiny, 0.0};
    const cplx l = cdiv(W[(int64_t)(k + 1) * m + k], d);
    __syncthreads();
    for (int c = k + 1 + lane; c < m; c += 64)
      W[(int64_t)(k + 1) * m + c] = csub(W[(int64_t)(k + 1) * m + c], cmul(l, W[(int64_t)k * m + c]));
    if (lane == 0) W[(int64_t)(k + 1) * m + k] = l;  // store multiplier
    __syncthreads();
  }
  for (int it = 0; it < 2; ++it) {
    // forward: apply pivots and multipliers to b
    if (lane == 0) {
      for (int k = 0; k < m - 1; ++k) {
        if (piv[k]) {
          const cplx t = b[k];
          b[k] = b[k + 1];
          b[k + 1] = t;
        }
        b[k + 1] = csub(b[k + 1], cmul(W[(int64_t)(k + 1) * m + k], b[k]));
      }
    }
    __syncthreads();
    // back substitution, column oriented
    for (int i = m - 1; i >= 0; --i) {
      cplx d = W[(int64_t)i * m + i];
      if (cabs2(d) == 0.0) d = {tiny, 0.0};
      const cplx si = cdiv(b[i], d);
      __syncthreads();
      if (lane == 0) b[i] = si;
      for (int r = lane; r < i; r += 64) b[r] = csub(b[r], cmul(W[(int64_t)r * m + i], si));
      __syncthreads();
    }
    // normalize
    double nrm = 0.0;
    for (int r = 0; r < m; ++r) nrm += cabs2(b[r]);
    nrm = sqrt(nrm);
    __syncthreads();
    for (int r = lane; r < m; r += 64) b[r] = {b[r].re / nrm, b[r].im / nrm};
    __syncthreads();
  }
  for (int r = lane; r < m; r += 64) {
    vr[(int64_t)q * m + r] = b[r].re;
    vi[(int64_t)q * m + r] = b[r].im;
  }
}

}  // namespace

// Work layout (doubles) in `scratch`: H copy m*m | wr m | wi m | info (1 int)
hipError_t launch_hessenberg_values(hipStream_t s, double* Hwork, int m, double* wr, double* wi, int* info) {
  hqr_kernel<<<1, 64, 0, s>>>(Hwork, m, wr, wi, info);
  return hipGetLastError();
}

hipError_t launch_hessenberg_vectors(hipStream_t s, const double* H, int m, const double* lr, const double* li,
                                     int nsel, double* cwork, double* vr, double* vi) {
  if (m > 512) return hipErrorInvalidValue;
  cplx* W = reinterpret_cast<cplx*>(cwork);
  cplx* b = W + (int64_t)nsel * m * m;
  inviter_kernel<<<nsel, 64, 0, s>>>(H, m, lr, li, nsel, W, b, vr, vi);
  return hipGetLastError();
}

}  // namespace kv
