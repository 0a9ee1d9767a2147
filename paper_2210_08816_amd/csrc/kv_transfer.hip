// Transfers between the packed staggered state and cell-centred fields on a
// (coarser, or differently clustered) network grid: the training targets of
// the learned Newton guess and the way its prediction becomes a state.
#include "kv_internal.h"

namespace kv {
namespace {

constexpr int XT = 256;

// Cell-centre values of a packed state X at fine cell (i, j, k):
// u, v, w averaged from their two faces (walls carry 0), theta = T - (1/2 - x_c).
struct CentreVals {
  const double* X;
  Grid g;
  __device__ void at(int i, int j, int k, double v[4]) const {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const double* U = X + g.ou;
    const double* Vv = X + g.ov;
    const double* W = X + g.ow;
    const double* T = X + g.oT;
    const int64_t rowu = ((int64_t)k * ny + j) * (nx - 1);
    const double ul = i > 0 ? U[rowu + i - 1] : 0.0;
    const double ur = i < nx - 1 ? U[rowu + i] : 0.0;
    const int64_t rowv = (int64_t)k * (ny - 1);
    const double vl = j > 0 ? Vv[(rowv + j - 1) * nx + i] : 0.0;
    const double vr = j < ny - 1 ? Vv[(rowv + j) * nx + i] : 0.0;
    const double wl = k > 0 ? W[((int64_t)(k - 1) * ny + j) * nx + i] : 0.0;
    const double wr = k < nz - 1 ? W[((int64_t)k * ny + j) * nx + i] : 0.0;
    v[0] = 0.5 * (ul + ur);
    v[1] = 0.5 * (vl + vr);
    v[2] = 0.5 * (wl + wr);
    v[3] = T[((int64_t)k * ny + j) * nx + i] - (0.5 - g.ax[0].c[i]);
  }
};

struct Affine {
  double shift[4], scale[4];
};

// out[c][K][J][I] = (volume average over the f^3 fine cells of coarse cell
// (I, J, K) of the centre value of channel c - shift[c]) / scale[c]
__global__ void __launch_bounds__(XT) cells_from_state_kernel(CentreVals cv, int f, Affine af, float* __restrict__ out) {
  const int rx = cv.g.nx / f, ry = cv.g.ny / f, rz = cv.g.nz / f;
  const int64_t nc = (int64_t)rx * ry * rz;
  for (int64_t e = (int64_t)blockIdx.x * XT + threadIdx.x; e < nc; e += (int64_t)gridDim.x * XT) {
    const int I = (int)(e % rx), J = (int)((e / rx) % ry), K = (int)(e / ((int64_t)rx * ry));
    double s[4] = {0, 0, 0, 0}, vol = 0.0;
    for (int dk = 0; dk < f; ++dk)
      for (int dj = 0; dj < f; ++dj)
        for (int di = 0; di < f; ++di) {
          const int i = I * f + di, j = J * f + dj, k = K * f + dk;
          const double wv = cv.g.ax[0].h[i] * cv.g.ax[1].h[j] * cv.g.ax[2].h[k];
          double v[4];
          cv.at(i, j, k, v);
#pragma unroll
          for (int c = 0; c < 4; ++c) s[c] += wv * v[c];
          vol += wv;
        }
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c * nc + e] = (float)((s[c] / vol - af.shift[c]) / af.scale[c]);
  }
}

// Interpolation tables of one axis: for every face (n+1) and every centre (n)
// of the solver grid, the lower node index q in the extended node list
// [0, c_0 .. c_{r-1}, 1] of the network grid and the weight t of node q+1.
struct Tables {
  const int* qf[3];
  const double* tf[3];
  const int* qc[3];
  const double* tc[3];
  int r[3];
};

// physical value of channel c at extended node (qx, qy, qz): walls carry
// velocity 0; theta is 0 on the x walls (T there is 1/2 - x) and continued
// from the adjacent cell on the adiabatic y and z walls
__device__ __forceinline__ double node_value(const float* __restrict__ cells, const Tables& tb, const Affine& af,
                                             int c, int qx, int qy, int qz) {
  const int rx = tb.r[0], ry = tb.r[1], rz = tb.r[2];
  const bool wx = qx == 0 || qx == rx + 1;
  const bool wy = qy == 0 || qy == ry + 1;
  const bool wz = qz == 0 || qz == rz + 1;
  if (c < 3) {
    if (wx || wy || wz) return 0.0;
  } else if (wx) {
    return 0.0;
  }
  const int i = qx - 1;
  const int j = min(max(qy - 1, 0), ry - 1);
  const int k = min(max(qz - 1, 0), rz - 1);
  const int64_t nc = (int64_t)rx * ry * rz;
  return af.shift[c] + af.scale[c] * (double)cells[c * nc + ((int64_t)k * ry + j) * rx + i];
}

__device__ __forceinline__ double trilinear(const float* __restrict__ cells, const Tables& tb, const Affine& af, int c,
                                            int qx, double tx, int qy, double ty, int qz, double tz) {
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int ax = d & 1, ay = (d >> 1) & 1, az = d >> 2;
    const double w = (ax ? tx : 1.0 - tx) * (ay ? ty : 1.0 - ty) * (az ? tz : 1.0 - tz);
    if (w != 0.0) s += w * node_value(cells, tb, af, c, qx + ax, qy + ay, qz + az);
  }
  return s;
}

// X = packed state whose every unknown is the trilinear interpolant of the
// network channels at its own position (faces for velocities, centres for T).
// INC: X += interpolant(cells) - interpolant(cells_ref) instead (the shift
// and the conduction profile cancel).
template <bool INC>
__global__ void __launch_bounds__(XT) state_from_cells_kernel(Grid g, const float* __restrict__ cells,
                                                            const float* __restrict__ cells_ref, Tables tb,
                                                            Affine af, double* __restrict__ X) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  for (int64_t e = (int64_t)blockIdx.x * XT + threadIdx.x; e < g.n; e += (int64_t)gridDim.x * XT) {
    int c, i, j, k;
    int64_t r;
    int px, py, pz;  // position kind per axis: 1 = face, 0 = centre
    if (e < g.ov) {
      c = 0;
      r = e - g.ou;
      i = (int)(r % (nx - 1)) + 1;
      j = (int)((r / (nx - 1)) % ny);
      k = (int)(r / ((int64_t)(nx - 1) * ny));
      px = 1, py = 0, pz = 0;
    } else if (e < g.ow) {
      c = 1;
      r = e - g.ov;
      i = (int)(r % nx);
      j = (int)((r / nx) % (ny - 1)) + 1;
      k = (int)(r / ((int64_t)nx * (ny - 1)));
      px = 0, py = 1, pz = 0;
    } else if (e < g.oT) {
      c = 2;
      r = e - g.ow;
      i = (int)(r % nx);
      j = (int)((r / nx) % ny);
      k = (int)(r / ((int64_t)nx * ny)) + 1;
      px = 0, py = 0, pz = 1;
    } else {
      c = 3;
      r = e - g.oT;
      i = (int)(r % nx);
      j = (int)((r / nx) % ny);
      k = (int)(r / ((int64_t)nx * ny));
      px = 0, py = 0, pz = 0;
    }
    const int qx = px ? tb.qf[0][i] : tb.qc[0][i];
    const double tx = px ? tb.tf[0][i] : tb.tc[0][i];
    const int qy = py ? tb.qf[1][j] : tb.qc[1][j];
    const double ty = py ? tb.tf[1][j] : tb.tc[1][j];
    const int qz = pz ? tb.qf[2][k] : tb.qc[2][k];
    const double tz = pz ? tb.tf[2][k] : tb.tc[2][k];
    const double v = trilinear(cells, tb, af, c, qx, tx, qy, ty, qz, tz);
    if (INC) {
      X[e] += v - trilinear(cells_ref, tb, af, c, qx, tx, qy, ty, qz, tz);
    } else {
      X[e] = c == 3 ? v + (0.5 - g.ax[0].c[i]) : v;
    }
  }
}

inline unsigned xblocks(int64_t n) {
  return (unsigned)std::min<int64_t>(16384, std::max<int64_t>(1, (n + XT - 1) / XT));
}

}  // namespace

hipError_t launch_cells_from_state(const kv_ctx* c, const double* X, int f, const double shift[4],
                                   const double scale[4], float* out) {
  Affine af;
  for (int q = 0; q < 4; ++q) af.shift[q] = shift[q], af.scale[q] = scale[q];
  const int64_t nc = (int64_t)(c->g.nx / f) * (c->g.ny / f) * (c->g.nz / f);
  cells_from_state_kernel<<<xblocks(nc), XT, 0, c->stream>>>(CentreVals{X, c->g}, f, af, out);
  return hipGetLastError();
}

hipError_t launch_state_from_cells(const kv_ctx* c, const float* cells, const float* cells_ref, const int r[3],
                                   const int* const q[6], const double* const t[6], const double shift[4],
                                   const double scale[4], double* X) {
  Affine af;
  for (int k = 0; k < 4; ++k) af.shift[k] = shift[k], af.scale[k] = scale[k];
  Tables tb;
  for (int a = 0; a < 3; ++a) {
    tb.qf[a] = q[2 * a];
    tb.qc[a] = q[2 * a + 1];
    tb.tf[a] = t[2 * a];
    tb.tc[a] = t[2 * a + 1];
    tb.r[a] = r[a];
  }
  if (cells_ref)
    state_from_cells_kernel<true><<<xblocks(c->g.n), XT, 0, c->stream>>>(c->g, cells, cells_ref, tb, af, X);
  else
    state_from_cells_kernel<false><<<xblocks(c->g.n), XT, 0, c->stream>>>(c->g, cells, nullptr, tb, af, X);
  return hipGetLastError();
}

}  // namespace kv
