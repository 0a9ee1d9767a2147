// Finite-volume stencils of the Boussinesq operator on the staggered grid.
//
// One thread per cell (i, j, k) produces every unknown that the cell owns:
// u on its west x-face (i >= 1), v on its south y-face (j >= 1), w on its
// bottom z-face (k >= 1) and T at its centre.  Threads of a block run along
// x, so all loads and stores are coalesced rows of the packed layout; the
// +-1 neighbours along y and z are re-read from the L1/L2 caches.
//
// The same kernel gives the Jacobian J(X0) x (paper Sec. 1: Newton and
// Arnoldi both act on it) and the steady right-hand side N(X) of Eqs. 1-2:
// every convective flux is a product (carrier velocity) x (carried
// quantity); J uses the product rule, N the product itself, which is the
// product-rule form with base = perturbation = X and a factor 1/2.
// Wall values: no-slip (velocities 0) at half-cell distance, T = +-1/2 on
// the x-walls for N (Eq. 4 in the centred variable), 0 for J, and no flux
// through the y- and z-walls (Eqs. 5-6).
#include <type_traits>

#include "kv_internal.h"

namespace kv {
namespace {

__device__ __forceinline__ double Uat(const double* __restrict__ X, const Grid& g, int i, int j, int k) {
  return (i <= 0 || i >= g.nx) ? 0.0 : X[g.ou + ((int64_t)k * g.ny + j) * (g.nx - 1) + (i - 1)];
}
__device__ __forceinline__ double Vat(const double* __restrict__ X, const Grid& g, int i, int j, int k) {
  return (j <= 0 || j >= g.ny) ? 0.0 : X[g.ov + ((int64_t)k * (g.ny - 1) + (j - 1)) * g.nx + i];
}
__device__ __forceinline__ double Wat(const double* __restrict__ X, const Grid& g, int i, int j, int k) {
  return (k <= 0 || k >= g.nz) ? 0.0 : X[g.ow + ((int64_t)(k - 1) * g.ny + j) * g.nx + i];
}
__device__ __forceinline__ double Tat(const double* __restrict__ X, const Grid& g, int i, int j, int k) {
  return X[g.oT + ((int64_t)k * g.ny + j) * g.nx + i];
}

// Fields straight from global memory (walls read as zero).
struct GlobalAcc {
  const Grid* g;
  const double* base;
  const double* pert;
  __device__ __forceinline__ const double* p(int s) const { return s ? pert : base; }
  __device__ __forceinline__ double U(int s, int i, int j, int k) const { return Uat(p(s), *g, i, j, k); }
  __device__ __forceinline__ double V(int s, int i, int j, int k) const { return Vat(p(s), *g, i, j, k); }
  __device__ __forceinline__ double W(int s, int i, int j, int k) const { return Wat(p(s), *g, i, j, k); }
  __device__ __forceinline__ double T(int s, int i, int j, int k) const { return Tat(p(s), *g, i, j, k); }
};

// Every unknown owned by cell (i, j, k).  MODE 0: y = J(base) pert.  MODE 1:
// y = N(pert) (base = pert).  A supplies the fields: A.U(s, i, j, k) etc. with
// s = 0 for the base flow and 1 for the perturbation, zero on walls.
// Outputs: plain stores (one-cell kernel) or raw buffer stores with 32-bit
// offsets (tiled kernel).
// face(c, v) hands the value of the cell's own face of component c (u, v,
// w) to an output that also forms the cell's net flux; a no-op otherwise.
struct PtrOut {
  double* y;
  __device__ __forceinline__ void put(int64_t idx, double v) const { y[idx] = v; }
  __device__ __forceinline__ void face(int, double) const {}
};
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
struct BufOut {
  __amdgpu_buffer_rsrc_t r;
  const Grid* g;
  __device__ __forceinline__ void put(int64_t idx, double v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)idx * 8, 0, 0);
  }
  __device__ __forceinline__ void face(int, double) const {}
};
// Buffer stores that also put the cell's low-face velocities into LDS
// (fl: u, v, w of the block's 256 cells; cleared beforehand, so a face the
// cell does not own, on a wall or outside the domain, reads as zero).  In
// LDS they occupy no registers while the rest of the point is computed.
// (Writing the zeros only where a cell owns no face, instead of clearing
// every plane, measured 3-5 us slower per 256^3 stencil.)
struct FaceOut : BufOut {
  double* fl;
  __device__ __forceinline__ void face(int c, double v) const { fl[c * 256 + threadIdx.x] = v; }
};

// The metrics one cell needs along one axis, held in registers: at the
// cell's low face f and high face f+1 (id = 1/centre gap, wl/wh =
// interpolation weights) and the widths of the cell and its low neighbour.
struct Met {
  double id0, id1, ih0, ihm, wl0, wh0, wl1, wh1;
};

__device__ __forceinline__ Met load_met(const Axis& A, int c) {
  Met m;
  const int n = A.n;
  const int cc = c < n ? c : n - 1;  // threads past the domain edge still load in range
  m.id0 = A.id[cc];
  m.id1 = A.id[cc + 1];
  m.ih0 = A.ih[cc];
  m.ihm = cc > 0 ? A.ih[cc - 1] : 0.0;
  m.wl0 = A.wlo[cc];
  m.wh0 = A.whi[cc];
  m.wl1 = A.wlo[cc + 1];
  m.wh1 = A.whi[cc + 1];
  return m;
}

// Quantities of a control volume's top z-face, carried up a column from
// plane k to plane k+1, where they are the bottom-face ones: the convective
// flux (f) and the diffusive gradient term (g) of u, v, w and T.  They are
// the same operands combined in the same order, so reusing them leaves every
// result bit-identical.  fresh: nothing carried (first plane of a march).
struct ZCarry {
  double uf, ug, vf, vg, wf, wg, tf, tg;
};

template <int MODE, class Acc, class Out>
__device__ __forceinline__ void point(const Grid& g, const Acc& A, int i, int j, int k, const Met& MX, const Met& MY,
                                      const Met& MZ, const Out& y, ZCarry& zc, bool fresh) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double s = MODE ? 0.5 : 1.0;
  const double TW = MODE ? 0.5 : 0.0, TE = MODE ? -0.5 : 0.0;

  // ---------------- u on x-face i ----------------
  if (i >= 1) {
    const double Uc = A.U(0, i, j, k), uc = A.U(1, i, j, k);
    const double Um = A.U(0, i - 1, j, k), um = A.U(1, i - 1, j, k);
    const double Up = A.U(0, i + 1, j, k), up = A.U(1, i + 1, j, k);
    // x: centre fluxes (u_bar)^2 at cells i (east) and i-1 (west)
    double adv = (0.5 * (Uc + Up) * (uc + up) - 0.5 * (Um + Uc) * (um + uc)) * MX.id0;
    const double xl = MX.wl0, xh = MX.wh0;
    // y: fluxes v_hat * u_hat at y-faces j and j+1 of the u control volume
    double fS = 0.0, fN = 0.0, uS = 0.0, uN = 0.0;
    if (j > 0) {
      const double yl = MY.wl0, yh = MY.wh0;
      const double UB = A.U(0, i, j - 1, k);
      uS = A.U(1, i, j - 1, k);
      const double Vh = xl * A.V(0, i - 1, j, k) + xh * A.V(0, i, j, k);
      const double vh = xl * A.V(1, i - 1, j, k) + xh * A.V(1, i, j, k);
      fS = Vh * (yl * uS + yh * uc) + vh * (yl * UB + yh * Uc);
    }
    if (j < ny - 1) {
      const double yl = MY.wl1, yh = MY.wh1;
      const double UB = A.U(0, i, j + 1, k);
      uN = A.U(1, i, j + 1, k);
      const double Vh = xl * A.V(0, i - 1, j + 1, k) + xh * A.V(0, i, j + 1, k);
      const double vh = xl * A.V(1, i - 1, j + 1, k) + xh * A.V(1, i, j + 1, k);
      fN = Vh * (yl * uc + yh * uN) + vh * (yl * Uc + yh * UB);
    }
    adv += (fN - fS) * MY.ih0;
    // z: fluxes w_hat * u_hat at z-faces k and k+1
    double fB = 0.0, fT = 0.0, gB, uT = 0.0;
    if (!fresh) {
      fB = zc.uf;
      gB = zc.ug;
    } else {
      double uB = 0.0;
      if (k > 0) {
        const double zl = MZ.wl0, zh = MZ.wh0;
        const double UB = A.U(0, i, j, k - 1);
        uB = A.U(1, i, j, k - 1);
        const double Wh = xl * A.W(0, i - 1, j, k) + xh * A.W(0, i, j, k);
        const double wh = xl * A.W(1, i - 1, j, k) + xh * A.W(1, i, j, k);
        fB = Wh * (zl * uB + zh * uc) + wh * (zl * UB + zh * Uc);
      }
      gB = (uc - uB) * MZ.id0;
    }
    if (k < nz - 1) {
      const double zl = MZ.wl1, zh = MZ.wh1;
      const double UB = A.U(0, i, j, k + 1);
      uT = A.U(1, i, j, k + 1);
      const double Wh = xl * A.W(0, i - 1, j, k + 1) + xh * A.W(0, i, j, k + 1);
      const double wh = xl * A.W(1, i - 1, j, k + 1) + xh * A.W(1, i, j, k + 1);
      fT = Wh * (zl * uc + zh * uT) + wh * (zl * Uc + zh * UB);
    }
    adv += (fT - fB) * MZ.ih0;
    const double gT = (uT - uc) * MZ.id1;
    zc.uf = fT;
    zc.ug = gT;
    double lap = ((up - uc) * MX.ih0 - (uc - um) * MX.ihm) * MX.id0;
    lap += ((uN - uc) * MY.id1 - (uc - uS) * MY.id0) * MY.ih0;
    lap += (gT - gB) * MZ.ih0;
    const double r = -s * adv + g.nu * lap;
    y.put(g.ou + ((int64_t)k * ny + j) * (nx - 1) + (i - 1), r);
    y.face(0, r);
  }

  // ---------------- v on y-face j ----------------
  if (j >= 1) {
    const double Vc = A.V(0, i, j, k), vc = A.V(1, i, j, k);
    const double Vm = A.V(0, i, j - 1, k), vm = A.V(1, i, j - 1, k);
    const double Vp = A.V(0, i, j + 1, k), vp = A.V(1, i, j + 1, k);
    double adv = (0.5 * (Vc + Vp) * (vc + vp) - 0.5 * (Vm + Vc) * (vm + vc)) * MY.id0;
    const double yl = MY.wl0, yh = MY.wh0;
    double fW = 0.0, fE = 0.0, vW = 0.0, vE = 0.0;
    if (i > 0) {
      const double xl = MX.wl0, xh = MX.wh0;
      const double VB = A.V(0, i - 1, j, k);
      vW = A.V(1, i - 1, j, k);
      const double Uh = yl * A.U(0, i, j - 1, k) + yh * A.U(0, i, j, k);
      const double uh = yl * A.U(1, i, j - 1, k) + yh * A.U(1, i, j, k);
      fW = Uh * (xl * vW + xh * vc) + uh * (xl * VB + xh * Vc);
    }
    if (i < nx - 1) {
      const double xl = MX.wl1, xh = MX.wh1;
      const double VB = A.V(0, i + 1, j, k);
      vE = A.V(1, i + 1, j, k);
      const double Uh = yl * A.U(0, i + 1, j - 1, k) + yh * A.U(0, i + 1, j, k);
      const double uh = yl * A.U(1, i + 1, j - 1, k) + yh * A.U(1, i + 1, j, k);
      fE = Uh * (xl * vc + xh * vE) + uh * (xl * Vc + xh * VB);
    }
    adv += (fE - fW) * MX.ih0;
    double fB = 0.0, fT = 0.0, gB, vT = 0.0;
    if (!fresh) {
      fB = zc.vf;
      gB = zc.vg;
    } else {
      double vB = 0.0;
      if (k > 0) {
        const double zl = MZ.wl0, zh = MZ.wh0;
        const double VB = A.V(0, i, j, k - 1);
        vB = A.V(1, i, j, k - 1);
        const double Wh = yl * A.W(0, i, j - 1, k) + yh * A.W(0, i, j, k);
        const double wh = yl * A.W(1, i, j - 1, k) + yh * A.W(1, i, j, k);
        fB = Wh * (zl * vB + zh * vc) + wh * (zl * VB + zh * Vc);
      }
      gB = (vc - vB) * MZ.id0;
    }
    if (k < nz - 1) {
      const double zl = MZ.wl1, zh = MZ.wh1;
      const double VB = A.V(0, i, j, k + 1);
      vT = A.V(1, i, j, k + 1);
      const double Wh = yl * A.W(0, i, j - 1, k + 1) + yh * A.W(0, i, j, k + 1);
      const double wh = yl * A.W(1, i, j - 1, k + 1) + yh * A.W(1, i, j, k + 1);
      fT = Wh * (zl * vc + zh * vT) + wh * (zl * Vc + zh * VB);
    }
    adv += (fT - fB) * MZ.ih0;
    const double gT = (vT - vc) * MZ.id1;
    zc.vf = fT;
    zc.vg = gT;
    double lap = ((vp - vc) * MY.ih0 - (vc - vm) * MY.ihm) * MY.id0;
    lap += ((vE - vc) * MX.id1 - (vc - vW) * MX.id0) * MX.ih0;
    lap += (gT - gB) * MZ.ih0;
    const double r = -s * adv + g.nu * lap;
    y.put(g.ov + ((int64_t)k * (ny - 1) + (j - 1)) * nx + i, r);
    y.face(1, r);
  }

  // ---------------- w on z-face k ----------------
  if (k >= 1) {
    const double Wc = A.W(0, i, j, k), wc = A.W(1, i, j, k);
    const double Wp = A.W(0, i, j, k + 1), wp = A.W(1, i, j, k + 1);
    // centre fluxes (w_bar)^2 and gradients at cells k (top) and k-1 (bottom);
    // the face k-1 below holds a w only for k >= 2
    const bool wfresh = fresh || k == 1;
    double cB, gB;
    if (!wfresh) {
      cB = zc.wf;
      gB = zc.wg;
    } else {
      const double Wm = A.W(0, i, j, k - 1), wm = A.W(1, i, j, k - 1);
      cB = 0.5 * (Wm + Wc) * (wm + wc);
      gB = (wc - wm) * MZ.ihm;
    }
    const double cT = 0.5 * (Wc + Wp) * (wc + wp), gT = (wp - wc) * MZ.ih0;
    zc.wf = cT;
    zc.wg = gT;
    double adv = (cT - cB) * MZ.id0;
    const double zl = MZ.wl0, zh = MZ.wh0;
    double fW = 0.0, fE = 0.0, wW = 0.0, wE = 0.0;
    if (i > 0) {
      const double xl = MX.wl0, xh = MX.wh0;
      const double WB = A.W(0, i - 1, j, k);
      wW = A.W(1, i - 1, j, k);
      const double Uh = zl * A.U(0, i, j, k - 1) + zh * A.U(0, i, j, k);
      const double uh = zl * A.U(1, i, j, k - 1) + zh * A.U(1, i, j, k);
      fW = Uh * (xl * wW + xh * wc) + uh * (xl * WB + xh * Wc);
    }
    if (i < nx - 1) {
      const double xl = MX.wl1, xh = MX.wh1;
      const double WB = A.W(0, i + 1, j, k);
      wE = A.W(1, i + 1, j, k);
      const double Uh = zl * A.U(0, i + 1, j, k - 1) + zh * A.U(0, i + 1, j, k);
      const double uh = zl * A.U(1, i + 1, j, k - 1) + zh * A.U(1, i + 1, j, k);
      fE = Uh * (xl * wc + xh * wE) + uh * (xl * Wc + xh * WB);
    }
    adv += (fE - fW) * MX.ih0;
    double fS = 0.0, fN = 0.0, wS = 0.0, wN = 0.0;
    if (j > 0) {
      const double yl = MY.wl0, yh = MY.wh0;
      const double WB = A.W(0, i, j - 1, k);
      wS = A.W(1, i, j - 1, k);
      const double Vh = zl * A.V(0, i, j, k - 1) + zh * A.V(0, i, j, k);
      const double vh = zl * A.V(1, i, j, k - 1) + zh * A.V(1, i, j, k);
      fS = Vh * (yl * wS + yh * wc) + vh * (yl * WB + yh * Wc);
    }
    if (j < ny - 1) {
      const double yl = MY.wl1, yh = MY.wh1;
      const double WB = A.W(0, i, j + 1, k);
      wN = A.W(1, i, j + 1, k);
      const double Vh = zl * A.V(0, i, j + 1, k - 1) + zh * A.V(0, i, j + 1, k);
      const double vh = zl * A.V(1, i, j + 1, k - 1) + zh * A.V(1, i, j + 1, k);
      fN = Vh * (yl * wc + yh * wN) + vh * (yl * Wc + yh * WB);
    }
    adv += (fN - fS) * MY.ih0;
    double lap = (gT - gB) * MZ.id0;
    lap += ((wE - wc) * MX.id1 - (wc - wW) * MX.id0) * MX.ih0;
    lap += ((wN - wc) * MY.id1 - (wc - wS) * MY.id0) * MY.ih0;
    const double buoy = zl * A.T(1, i, j, k - 1) + zh * A.T(1, i, j, k);
    const double r = -s * adv + g.nu * lap + g.beta * buoy;
    y.put(g.ow + ((int64_t)(k - 1) * ny + j) * nx + i, r);
    y.face(2, r);
  }

  // ---------------- T at the cell centre ----------------
  {
    const double Tb = A.T(0, i, j, k), tc = A.T(1, i, j, k);
    double adv = 0.0, lap = 0.0;
    // x
    {
      double fW = 0.0, fE = 0.0;
      const double tW = (i > 0) ? A.T(1, i - 1, j, k) : TW;
      const double tE = (i < nx - 1) ? A.T(1, i + 1, j, k) : TE;
      if (i > 0) {
        const double xl = MX.wl0, xh = MX.wh0;
        const double Th = xl * A.T(0, i - 1, j, k) + xh * Tb;
        fW = A.U(0, i, j, k) * (xl * tW + xh * tc) + A.U(1, i, j, k) * Th;
      }
      if (i < nx - 1) {
        const double xl = MX.wl1, xh = MX.wh1;
        const double Th = xl * Tb + xh * A.T(0, i + 1, j, k);
        fE = A.U(0, i + 1, j, k) * (xl * tc + xh * tE) + A.U(1, i + 1, j, k) * Th;
      }
      adv += (fE - fW) * MX.ih0;
      lap += ((tE - tc) * MX.id1 - (tc - tW) * MX.id0) * MX.ih0;
    }
    // y
    {
      double fS = 0.0, fN = 0.0, gS = 0.0, gN = 0.0;
      if (j > 0) {
        const double yl = MY.wl0, yh = MY.wh0;
        const double tS = A.T(1, i, j - 1, k);
        const double Th = yl * A.T(0, i, j - 1, k) + yh * Tb;
        fS = A.V(0, i, j, k) * (yl * tS + yh * tc) + A.V(1, i, j, k) * Th;
        gS = (tc - tS) * MY.id0;
      }
      if (j < ny - 1) {
        const double yl = MY.wl1, yh = MY.wh1;
        const double tN = A.T(1, i, j + 1, k);
        const double Th = yl * Tb + yh * A.T(0, i, j + 1, k);
        fN = A.V(0, i, j + 1, k) * (yl * tc + yh * tN) + A.V(1, i, j + 1, k) * Th;
        gN = (tN - tc) * MY.id1;
      }
      adv += (fN - fS) * MY.ih0;
      lap += (gN - gS) * MY.ih0;
    }
    // z
    {
      double fB = 0.0, fT = 0.0, gB = 0.0, gT = 0.0;
      if (!fresh) {
        fB = zc.tf;
        gB = zc.tg;
      } else if (k > 0) {
        const double zl = MZ.wl0, zh = MZ.wh0;
        const double tB = A.T(1, i, j, k - 1);
        const double Th = zl * A.T(0, i, j, k - 1) + zh * Tb;
        fB = A.W(0, i, j, k) * (zl * tB + zh * tc) + A.W(1, i, j, k) * Th;
        gB = (tc - tB) * MZ.id0;
      }
      if (k < nz - 1) {
        const double zl = MZ.wl1, zh = MZ.wh1;
        const double tT = A.T(1, i, j, k + 1);
        const double Th = zl * Tb + zh * A.T(0, i, j, k + 1);
        fT = A.W(0, i, j, k + 1) * (zl * tc + zh * tT) + A.W(1, i, j, k + 1) * Th;
        gT = (tT - tc) * MZ.id1;
      }
      adv += (fT - fB) * MZ.ih0;
      lap += (gT - gB) * MZ.ih0;
      zc.tf = fT;
      zc.tg = gT;
    }
    y.put(g.oT + ((int64_t)k * ny + j) * nx + i, -s * adv + g.kappa * lap);
  }
}


// One thread per cell, fields from global memory (kept for very small grids).
template <int MODE>
__global__ void __launch_bounds__(256) operator_kernel(Grid g, const double* __restrict__ B,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  GlobalAcc A{&g, B, x};
  ZCarry zc;
  point<MODE>(g, A, i, j, k, load_met(g.ax[0], i), load_met(g.ax[1], j), load_met(g.ax[2], k), PtrOut{y}, zc, true);
}

// ---- 2.5-D tiled version ---------------------------------------------------------
// A block owns a TX x TY tile of (x, y) columns and a chunk of kc z-planes.  It
// marches up in z with the planes the stencil reaches (k-1, k, k+1), a
// one-cell halo in x and y, in LDS and registers; each plane is loaded once,
// as coalesced x-rows, and every output row is written once.
constexpr int TX = 64, TY = 4;
static_assert(TX * TY == 256, "one tile cell per thread of a 256-thread block (FaceOut's LDS slots)");
constexpr int PX = TX + 2, PY = TY + 2, PLANE = PX * PY;

// LDS holds only what other columns read: every field on plane k; u and v
// also on plane k-1 (the w equation reads u(i+1, k-1), v(j+1, k-1)); w also
// on plane k+1 (the u and v equations read w(i-1, k+1), w(j-1, k+1)).  The
// thread's own column at k-1 (w, T) and k+1 (u, v, T) is kept in registers.
// That is 7 planes per field set (14 for J, 7 for N) instead of a 3-plane
// ring of every field: 44 KB per block for J, so three blocks share a CU.
template <int NF>
struct TileAcc {
  static constexpr int NSF = NF / 4;  // field sets: base and perturbation (J) or one (N)
  const double* lds;
  int ic, jc, kc, off;                // this thread's cell and its offset inside a plane
  double un[NSF], vn[NSF], tn[NSF];   // own column, plane k+1
  double wp[NSF], tp[NSF];            // own column, plane k-1
  // LDS plane of (component, set, plane parity): u, v, w two planes each, T one
  static __device__ __forceinline__ int slot(int comp, int s, int pp) {
    return comp < 3 ? (comp * NSF + s) * 2 + pp : 6 * NSF + s;
  }
  __device__ __forceinline__ double ld(int comp, int s, int k, int i, int j) const {
    return lds[slot(comp, s, k & 1) * PLANE + off + (j - jc) * PX + (i - ic)];
  }
  __device__ __forceinline__ int st(int s) const { return NSF == 2 ? s : 0; }
  __device__ __forceinline__ double U(int s, int i, int j, int k) const {
    return k > kc ? un[st(s)] : ld(0, st(s), k, i, j);
  }
  __device__ __forceinline__ double V(int s, int i, int j, int k) const {
    return k > kc ? vn[st(s)] : ld(1, st(s), k, i, j);
  }
  __device__ __forceinline__ double W(int s, int i, int j, int k) const {
    return k < kc ? wp[st(s)] : ld(2, st(s), k, i, j);
  }
  __device__ __forceinline__ double T(int s, int i, int j, int k) const {
    return k > kc ? tn[st(s)] : (k < kc ? tp[st(s)] : ld(3, st(s), k, i, j));
  }
};

// A plane of every field, fetched into registers: entry 0 of each thread is
// its own column, entry 1 (the first 140 threads) one of the 140 halo
// columns around the 64 x 4 tile.  Outside the domain and on walls the value
// is zero.
constexpr int NHALO = 2 * PX + 2 * TY;

template <int NF>
struct PlaneRegs {
  double v[NF][2];
};

// Where this thread's two entries live in each packed block, once per
// block: a plane kp of block c is at  base[c][q] + kp * stride[c]  (32-bit
// offsets: n < 2^31), valid where the in-plane position lies in the block;
// pos[q] is the entry's position in an LDS plane (-1: none).
struct FetchMap {
  int32_t base[4][2];
  int32_t stride[4];
  uint32_t ok[2];  // bit c: in-plane position valid for block c
  int pos[2];
};

__device__ __forceinline__ FetchMap fetch_map(const Grid& g, int i0, int j0) {
  FetchMap m;
  const int nx = g.nx, ny = g.ny;
  m.stride[0] = ny * (nx - 1);
  m.stride[1] = (ny - 1) * nx;
  m.stride[2] = ny * nx;
  m.stride[3] = ny * nx;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int ti, tj;
    bool rin = true;
    if (q == 0) {
      ti = threadIdx.x % TX;
      tj = threadIdx.x / TX;
    } else {
      const int h = threadIdx.x;
      rin = h < NHALO;
      if (h < PX) {
        ti = h - 1, tj = -1;
      } else if (h < 2 * PX) {
        ti = h - PX - 1, tj = TY;
      } else if (h < 2 * PX + TY) {
        ti = -1, tj = h - 2 * PX;
      } else {
        ti = TX, tj = h - 2 * PX - TY;
      }
    }
    const int i = i0 + ti, j = j0 + tj;
    m.pos[q] = rin ? (tj + 1) * PX + (ti + 1) : -1;
    const bool iin = i >= 0 && i < nx, jin = j >= 0 && j < ny;
    uint32_t ok = 0;
    if (rin && jin && i >= 1 && i <= nx - 1) ok |= 1u;
    if (rin && iin && j >= 1 && j <= ny - 1) ok |= 2u;
    if (rin && iin && jin) ok |= 4u | 8u;
    m.ok[q] = ok;
    m.base[0][q] = (int32_t)g.ou + j * (nx - 1) + (i - 1);
    m.base[1][q] = (int32_t)g.ov + (j - 1) * nx + i;
    m.base[2][q] = (int32_t)g.ow + (j - ny) * nx + i;  // w plane kp is stored as kp - 1
    m.base[3][q] = (int32_t)g.oT + j * nx + i;
  }
  return m;
}

// A raw buffer over one packed vector: loads past num_records return 0, so
// wall and out-of-domain tile entries need no branch.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const double* p, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, (int)(n * 8), 0x00020000);
}
constexpr int OOB = 0x7ffffff8;  // a byte offset past every buffer

// field f of a PlaneRegs: component f / NSF, set f % NSF
template <int NF>
__device__ __forceinline__ void fetch_plane(const Grid& g, __amdgpu_buffer_rsrc_t rB, __amdgpu_buffer_rsrc_t rx,
                                            const FetchMap& m, int kp, PlaneRegs<NF>& R) {
  constexpr int NSF = NF / 4;
  // plane validity per block: u, v, T need 0 <= kp < nz; w (faces) 1 <= kp <= nz-1
  const bool kin = (kp >= 0 && kp < g.nz);
  const bool win = (kp >= 1 && kp < g.nz);
  // waves none of whose lanes holds a halo column skip the halo loads
  const bool halo_wave = (int)(threadIdx.x >> 6) <= (NHALO - 1) / 64;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (q == 1 && !halo_wave) break;
    int off[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const bool valid = ((m.ok[q] >> c) & 1u) && (c == 2 ? win : kin);
      off[c] = valid ? (m.base[c][q] + kp * m.stride[c]) * 8 : OOB;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int comp = f / NSF;
      const __amdgpu_buffer_rsrc_t r = (NSF == 2 && (f % NSF) == 0) ? rB : rx;
      R.v[f][q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off[comp], 0, 0));
    }
  }
}

// Store the components in mask (bit c: component c) of plane kp.
template <int NF>
__device__ __forceinline__ void store_plane(double* lds, const FetchMap& m, int kp, unsigned mask,
                                            const PlaneRegs<NF>& R) {
  constexpr int NSF = NF / 4;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (m.pos[q] < 0) continue;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int comp = f / NSF, s = f % NSF;
      if ((mask >> comp) & 1u) lds[TileAcc<NF>::slot(comp, s, kp & 1) * PLANE + m.pos[q]] = R.v[f][q];
    }
  }
}

// DIV: the kernel also writes the net face flux of y over each cell into dv
// (the divergence that the projection starts from, Eq. 2 integrated over
// the cell), scaled by V^-1/2 like scaled_divergence_kernel.  A cell's own
// faces are the low ones it computes; its high faces come from the next
// lane (u), from the next wave through LDS (v) and from the next plane of
// the march (w).  Where that neighbour lies in another block (the last
// column of a tile, its last row, the last plane of a z-chunk) the cell
// gets its partial net flux over its volume, unscaled, which
// divergence_edges_kernel completes.
template <int MODE, bool DIV>
__device__ __forceinline__ void operator_tiled_body(const Grid& g, const double* __restrict__ B,
                                                    const double* __restrict__ x, double* __restrict__ y,
                                                    int tiles_x, int tiles_y, int chunks, int kc,
                                                    double* __restrict__ dv) {
  constexpr int NF = MODE ? 4 : 8;
  constexpr int NSF = NF / 4;
  extern __shared__ double lds[];
  // XCD-aware order: blocks are dealt round-robin over 8 XCDs; give each XCD a
  // contiguous range of tiles so y-neighbouring tiles share an L2.
  const int64_t total = (int64_t)tiles_x * tiles_y * chunks;
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t w = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (w >= total) return;
  const int bx = (int)(w % tiles_x);
  const int by = (int)((w / tiles_x) % tiles_y);
  const int bz = (int)(w / ((int64_t)tiles_x * tiles_y));
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * kc;
  const int k1 = min(g.nz, k0 + kc);
  // a wave is one x-row of the tile (TX = 64), so j is uniform per wave
  static_assert(TX == 64, "one wave per tile row");
  const int i = i0 + (threadIdx.x % TX), j = __builtin_amdgcn_readfirstlane(j0 + (int)(threadIdx.x / TX));
  const Met MX = load_met(g.ax[0], i), MY = load_met(g.ax[1], j);
  ZCarry zc;
  const FetchMap fm = fetch_map(g, i0, j0);
  const __amdgpu_buffer_rsrc_t rB = vec_rsrc(B, g.n), rx = vec_rsrc(x, g.n);
  // DIV: the faces of the block's cells in LDS, and there too the net flux
  // over the volume of each thread's cell below, less its top face's term
  double* fl = lds + (MODE ? 7 : 14) * PLANE;
  typename std::conditional<DIV, FaceOut, BufOut>::type out;
  out.r = vec_rsrc(y, g.n);
  out.g = &g;
  if constexpr (DIV) out.fl = fl;
  const int lane = threadIdx.x % TX, row = threadIdx.x / TX;
  const bool ex = lane == TX - 1 && i + 1 < g.nx, ey = row == TY - 1 && j + 1 < g.ny;
  const __amdgpu_buffer_rsrc_t rd = vec_rsrc(dv, (int64_t)g.nx * g.ny * g.nz);
  // the column's sqrt(h_x), read back from LDS (fl[1024 + lane]) where it is
  // used rather than held in registers
  if (DIV && row == 0) fl[1024 + lane] = g.ax[0].sq[min(i, g.nx - 1)];
  // cell (i, j, kk) of dv: V^-1/2 (net flux) = sqrt(V) (net flux / V), or the
  // partial net flux / V on tile edges
  auto emit = [&](int kk, double net) {
    if (i >= g.nx || j >= g.ny) return;
    const bool edge = ex || ey || (kk == k1 - 1 && k1 < g.nz);
    const double v = edge ? net : net * (fl[1024 + lane] * g.ax[1].sq[j] * g.ax[2].sq[kk]);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rd, ((kk * g.ny + j) * g.nx + i) * 8, 0, 0);
  };
  TileAcc<NF> A;
  A.lds = lds;
  A.ic = i;
  A.jc = j;
  A.off = (j - j0 + 1) * PX + (i - i0 + 1);
  // prologue: u, v of plane k0-1 and w, T of it in registers; every field of
  // plane k0; w of plane k0+1 (u, v, T of it in registers)
  PlaneRegs<NF> Rn, Rf;
  fetch_plane<NF>(g, rB, rx, fm, k0 - 1, Rf);
  fetch_plane<NF>(g, rB, rx, fm, k0, Rn);
  store_plane<NF>(lds, fm, k0 - 1, 0x3u, Rf);
#pragma unroll
  for (int s = 0; s < NSF; ++s) {
    A.wp[s] = Rf.v[2 * NSF + s][0];
    A.tp[s] = Rf.v[3 * NSF + s][0];
  }
  store_plane<NF>(lds, fm, k0, 0xfu, Rn);
  fetch_plane<NF>(g, rB, rx, fm, k0 + 1, Rn);
  store_plane<NF>(lds, fm, k0 + 1, 0x4u, Rn);
  __syncthreads();
  for (int k = k0; k < k1; ++k) {
    // software pipeline: plane k+2 is in flight while plane k is computed
    const bool more = k + 1 < k1;
    if (more) fetch_plane<NF>(g, rB, rx, fm, k + 2, Rf);
#pragma unroll
    for (int s = 0; s < NSF; ++s) {
      A.un[s] = Rn.v[0 * NSF + s][0];
      A.vn[s] = Rn.v[1 * NSF + s][0];
      A.tn[s] = Rn.v[3 * NSF + s][0];
    }
    A.kc = k;
    double wk[NSF], tk[NSF];
#pragma unroll
    for (int s = 0; s < NSF; ++s) {
      wk[s] = A.ld(2, s, k, i, j);
      tk[s] = A.ld(3, s, k, i, j);
    }
    if constexpr (DIV) fl[threadIdx.x] = fl[256 + threadIdx.x] = fl[512 + threadIdx.x] = 0.0;
    if (i < g.nx && j < g.ny) point<MODE>(g, A, i, j, k, MX, MY, load_met(g.ax[2], k), out, zc, k == k0);
    __syncthreads();
    if (more) {
      // u, v, T of plane k+1 replace those of planes k-1 and k; w of plane
      // k+2 replaces w of plane k
      store_plane<NF>(lds, fm, k + 1, 0xbu, Rn);
      store_plane<NF>(lds, fm, k + 2, 0x4u, Rf);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        Rn.v[f][0] = Rf.v[f][0];
        Rn.v[f][1] = Rf.v[f][1];
      }
#pragma unroll
      for (int s = 0; s < NSF; ++s) {
        A.wp[s] = wk[s];
        A.tp[s] = tk[s];
      }
    }
    if constexpr (DIV) {
      // (after the plane shift, where the fewest registers are live) u on
      // the east face is the next lane's own (zero past the domain or on
      // the tile's last column), v on the north face the next row's
      const int t = threadIdx.x;
      const double uo = fl[t], uh = lane < TX - 1 ? fl[t + 1] : 0.0;
      const double vo = fl[256 + t], vh = row < TY - 1 ? fl[256 + t + TX] : 0.0;
      const double wo = fl[512 + t];
      // the carry lives in LDS between iterations (fl[768 + t], own slot)
      if (k > k0) emit(k - 1, fl[768 + t] + wo * g.ax[2].ih[k - 1]);
      fl[768 + t] = (uh - uo) * MX.ih0 + (vh - vo) * MY.ih0 - wo * g.ax[2].ih[k];
    }
    __syncthreads();
  }
  // the chunk's last cell: its top face is the wall (w = 0) or the next
  // chunk's first plane
  if constexpr (DIV) emit(k1 - 1, fl[768 + threadIdx.x]);
}

template <int MODE>
__global__ void __launch_bounds__(256) operator_tiled_kernel(Grid g, const double* __restrict__ B,
                                                             const double* __restrict__ x, double* __restrict__ y,
                                                             int tiles_x, int tiles_y, int chunks, int kc) {
  operator_tiled_body<MODE, false>(g, B, x, y, tiles_x, tiles_y, chunks, kc, nullptr);
}

// y = J(X0) x with the scaled divergence of y in dv.  Three waves per SIMD
// (at most 168 VGPRs) are asked for explicitly: left alone, the compiler
// gives the fused kernel 174 and the CU only two blocks.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
operator_divergence_kernel(Grid g, const double* __restrict__ B, const double* __restrict__ x,
                           double* __restrict__ y, int tiles_x, int tiles_y, int chunks, int kc,
                           double* __restrict__ dv) {
  operator_tiled_body<0, true>(g, B, x, y, tiles_x, tiles_y, chunks, kc, dv);
}

// Column-marching kernels: a (64, 4) block owns a tile of (x, y) columns
// and a run of consecutive z-planes (the planes split evenly over gridDim.z:
// 16 per block on large grids, fewer on small ones so that enough blocks
// exist), and each thread walks up its column keeping
// the value its plane shares with the one below (w on the face between them,
// or p of the cell below) in a register, so that every input is read once.
__device__ __forceinline__ int march_planes(int nz) { return (nz + (int)gridDim.z - 1) / (int)gridDim.z; }

// out = V^{1/2} (D y) = (net outward face flux of the velocity) / sqrt(V_c)
template <typename OutT>
__global__ void __launch_bounds__(256) scaled_divergence_kernel(Grid g, const double* __restrict__ y,
                                                                OutT* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int kd = march_planes(g.nz);
  const int k0 = blockIdx.z * kd, k1 = min(g.nz, k0 + kd);
  const Axis& AX = g.ax[0];
  const Axis& AY = g.ax[1];
  const Axis& AZ = g.ax[2];
  const double hx = AX.h[i], hy = AY.h[j], sxy = AX.isq[i] * AY.isq[j];
  double wlo = Wat(y, g, i, j, k0);
#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    const double whi = Wat(y, g, i, j, k + 1);
    const double fx = Uat(y, g, i + 1, j, k) - Uat(y, g, i, j, k);
    const double fy = Vat(y, g, i, j + 1, k) - Vat(y, g, i, j, k);
    const double fz = whi - wlo;
    const double hz = AZ.h[k];
    const double net = hy * hz * fx + hx * hz * fy + hx * hy * fz;
    out[((int64_t)k * g.ny + j) * g.nx + i] = (OutT)(net * (sxy * AZ.isq[k]));
    wlo = whi;
  }
}

// The terms a tile-edge cell (i, j, k) lacks, added to its partial net flux
// over its volume, and the scaling by sqrt(V).
__device__ __forceinline__ double complete_edge(const Grid& g, const double* __restrict__ y, int kc, int i, int j,
                                                int k, double net) {
  const Axis& AX = g.ax[0];
  const Axis& AY = g.ax[1];
  const Axis& AZ = g.ax[2];
  if (i % 64 == 63 && i + 1 < g.nx) net += Uat(y, g, i + 1, j, k) * AX.ih[i];
  if (j % 4 == 3 && j + 1 < g.ny) net += Vat(y, g, i, j + 1, k) * AY.ih[j];
  if (k % kc == kc - 1 && k + 1 < g.nz) net += Wat(y, g, i, j, k + 1) * AZ.ih[k];
  return net * (AX.sq[i] * AY.sq[j] * AZ.sq[k]);
}

constexpr int EDGE_KQ = 4;  // planes per thread on the edge rows

// Completes the cells the fused stencil left with a partial net flux: adds
// u on the east face of a tile's last column (i = 64 m + 63), v on the north
// face of its last row (j = 4 m + 3), w on the top face of a z-chunk's last
// plane (k = kc m + kc - 1), each where that face is inside the domain, then
// scales by sqrt(V).  Three disjoint sets of blocks: every cell of the edge
// rows (b1 blocks: 256 cells of a row, EDGE_KQ consecutive planes each, all
// loads issued before any arithmetic: these cells are most of the work and
// the pass is bound by load latency), the edge columns' cells in the other
// rows (b2: 256 rows of a column), and the chunk-end planes' cells in neither
// (the rest: 256 cells of a row).  Block indices are split with wave-uniform
// arithmetic; cx and cy count the edge columns and rows.
__global__ void __launch_bounds__(256) divergence_edges_kernel(Grid g, const double* __restrict__ y,
                                                               double* __restrict__ dv, int kc, int cx, int cy,
                                                               unsigned b1, unsigned b2) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned nbx = (unsigned)(nx + 255) / 256, nby = (unsigned)(ny + 255) / 256;
  unsigned b = blockIdx.x;
  const int t = threadIdx.x;
  if (b < b1) {
    const int i = (int)(b % nbx) * 256 + t;
    b /= nbx;
    const int j = 4 * (int)(b % (unsigned)cy) + 3;
    const int k0 = EDGE_KQ * (int)(b / (unsigned)cy);
    if (i >= nx) return;
    const int64_t plane = (int64_t)ny * nx, c0 = ((int64_t)k0 * ny + j) * nx + i;
    const int64_t v0 = g.ov + ((int64_t)k0 * (ny - 1) + j) * nx + i;  // v on the north face at k0
    double net[EDGE_KQ], vn[EDGE_KQ];
#pragma unroll
    for (int r = 0; r < EDGE_KQ; ++r) {
      const bool in = k0 + r < nz;
      net[r] = in ? dv[c0 + r * plane] : 0.0;
      vn[r] = in ? y[v0 + (int64_t)r * (ny - 1) * nx] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < EDGE_KQ; ++r) {
      const int k = k0 + r;
      if (k >= nz) break;
      // the north face's term is added here from the loaded value; the other
      // two (east face, top face) where they apply
      double v = net[r] + vn[r] * g.ax[1].ih[j];
      if (i % 64 == 63 && i + 1 < nx) v += Uat(y, g, i + 1, j, k) * g.ax[0].ih[i];
      if (k % kc == kc - 1 && k + 1 < nz) v += Wat(y, g, i, j, k + 1) * g.ax[2].ih[k];
      dv[c0 + r * plane] = v * (g.ax[0].sq[i] * g.ax[1].sq[j] * g.ax[2].sq[k]);
    }
    return;
  }
  int i, j, k;
  if ((b -= b1) < b2) {
    i = 64 * (int)(b % (unsigned)cx) + 63;
    b /= (unsigned)cx;
    j = (int)(b % nby) * 256 + t;
    k = (int)(b / nby);
    if (j >= ny || (j % 4 == 3 && j + 1 < ny)) return;
  } else {
    b -= b2;
    i = (int)(b % nbx) * 256 + t;
    b /= nbx;
    j = (int)(b % (unsigned)ny);
    k = kc * (int)(b / (unsigned)ny) + kc - 1;
    if (i >= nx || (j % 4 == 3 && j + 1 < ny) || (i % 64 == 63 && i + 1 < nx)) return;
  }
  const int64_t cell = ((int64_t)k * ny + j) * nx + i;
  dv[cell] = complete_edge(g, y, kc, i, j, k, dv[cell]);  // dv: net flux / V, less the missing terms
}

__device__ __forceinline__ double fin_abs(double v);

// Mixed-form refinement sweep, fused: yout = yin - G p on the velocity, and
// from the corrected field (every face of the cell corrected locally from p,
// so no thread reads another's output) the net flux of the cell: its scaled
// value feeds the next sweep (bnext, FP32, optional) and block maxima of
// |net flux| and |face flux| give the normalized divergence.  T is not
// touched (the sweeps alternate between the caller's vector, whose T is
// final, and a scratch vector whose T is never read).  Threads march up
// z-columns like the divergence kernel; the corrected w on a cell's top face
// is the next plane's bottom one.
__global__ void __launch_bounds__(256) correct_divergence_kernel(Grid g, const double* __restrict__ yin,
                                                                 const float* __restrict__ p,
                                                                 double* __restrict__ yout,
                                                                 float* __restrict__ bnext,
                                                                 double* __restrict__ part) {
  __shared__ double s0[4], s1[4];
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t plane = (int64_t)nx * ny;
  double mb = 0.0, mf = 0.0;
  if (i < nx && j < ny) {
    const int kd = march_planes(nz);
    const int k0 = blockIdx.z * kd, k1 = min(nz, k0 + kd);
    const Axis& AX = g.ax[0];
    const Axis& AY = g.ax[1];
    const Axis& AZ = g.ax[2];
    const double idx0 = AX.id[i], idx1 = AX.id[i + 1], idy0 = AY.id[j], idy1 = AY.id[j + 1];
    const double hx = AX.h[i], hy = AY.h[j], sxy = AX.isq[i] * AY.isq[j];
    int64_t c = k0 * plane + (int64_t)j * nx + i;
    double pc = p[c];
    double w0 = 0.0;  // corrected w on the bottom face of the current cell
    if (k0 >= 1) w0 = Wat(yin, g, i, j, k0) - (pc - p[c - plane]) * AZ.id[k0];
    for (int k = k0; k < k1; ++k, c += plane) {
      double u0 = 0.0, u1 = 0.0, v0 = 0.0, v1 = 0.0, w1 = 0.0, pn = 0.0;
      if (i >= 1) {
        u0 = Uat(yin, g, i, j, k) - (pc - p[c - 1]) * idx0;
        yout[g.ou + ((int64_t)k * ny + j) * (nx - 1) + (i - 1)] = u0;
      }
      if (i + 1 <= nx - 1) u1 = Uat(yin, g, i + 1, j, k) - (p[c + 1] - pc) * idx1;
      if (j >= 1) {
        v0 = Vat(yin, g, i, j, k) - (pc - p[c - nx]) * idy0;
        yout[g.ov + ((int64_t)k * (ny - 1) + (j - 1)) * nx + i] = v0;
      }
      if (j + 1 <= ny - 1) v1 = Vat(yin, g, i, j + 1, k) - (p[c + nx] - pc) * idy1;
      if (k >= 1) yout[g.ow + ((int64_t)(k - 1) * ny + j) * nx + i] = w0;
      if (k + 1 <= nz - 1) {
        pn = p[c + plane];
        w1 = Wat(yin, g, i, j, k + 1) - (pn - pc) * AZ.id[k + 1];
      }
      const double hz = AZ.h[k];
      const double net = hy * hz * (u1 - u0) + hx * hz * (v1 - v0) + hx * hy * (w1 - w0);
      if (bnext) bnext[c] = (float)(net * (sxy * AZ.isq[k]));
      mb = fmax(mb, fin_abs(net));
      mf = fmax(mf, fmax(fin_abs(u0 * hy * hz), fmax(fin_abs(v0 * hx * hz), fin_abs(w0 * hx * hy))));
      w0 = w1;
      pc = pn;
    }
  }
  // wavefront maxima by lane exchange, then the 4 waves through LDS
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mb = fmax(mb, __shfl_xor(mb, o, 64));
    mf = fmax(mf, __shfl_xor(mf, o, 64));
  }
  if ((t & 63) == 0) {
    s0[t >> 6] = mb;
    s1[t >> 6] = mf;
  }
  __syncthreads();
  if (t == 0) {
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * blk] = fmax(fmax(s0[0], s0[1]), fmax(s0[2], s0[3]));
    part[2 * blk + 1] = fmax(fmax(s1[0], s1[1]), fmax(s1[2], s1[3]));
  }
}

// y_vel -= G p at the interior faces owned by cell (i, j, k), marching up
// the column (p of the cell below kept in a register)
__global__ void __launch_bounds__(256) gradient_correction_kernel(Grid g, const double* __restrict__ p,
                                                                  double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int kd = march_planes(g.nz);
  const int k0 = blockIdx.z * kd, k1 = min(g.nz, k0 + kd);
  if (k0 >= k1) return;
  const int nx = g.nx, ny = g.ny;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t su = (int64_t)(nx - 1) * ny, sv = (int64_t)(ny - 1) * nx;
  const double idx = g.ax[0].id[i], idy = g.ax[1].id[j];
  const bool du = i >= 1, dv = j >= 1;
  double* yu = y + g.ou;
  double* yv = y + g.ov;
  double* yw = y + g.ow;
  int64_t c = (int64_t)k0 * plane + (int64_t)j * nx + i;
  int64_t iu = (int64_t)k0 * su + (int64_t)j * (nx - 1) + (i - 1);
  int64_t iv = (int64_t)k0 * sv + (int64_t)(j - 1) * nx + i;
  int64_t iw = (int64_t)(k0 - 1) * plane + (int64_t)j * nx + i;
  // plane k's operands are loaded one plane ahead: the loads of plane k+1 are
  // issued before the stores of plane k (they touch other faces)
  double pm = k0 >= 1 ? p[c - plane] : 0.0;
  double pc = p[c], px = du ? p[c - 1] : 0.0, py = dv ? p[c - nx] : 0.0;
  double u = du ? yu[iu] : 0.0, v = dv ? yv[iv] : 0.0, w = k0 >= 1 ? yw[iw] : 0.0;
  for (int k = k0; k < k1; ++k) {
    double pc1 = 0.0, px1 = 0.0, py1 = 0.0, u1 = 0.0, v1 = 0.0, w1 = 0.0;
    if (k + 1 < k1) {
      pc1 = p[c + plane];
      if (du) {
        px1 = p[c + plane - 1];
        u1 = yu[iu + su];
      }
      if (dv) {
        py1 = p[c + plane - nx];
        v1 = yv[iv + sv];
      }
      w1 = yw[iw + plane];
    }
    if (du) yu[iu] = u - (pc - px) * idx;
    if (dv) yv[iv] = v - (pc - py) * idy;
    if (k >= 1) yw[iw] = w - (pc - pm) * g.ax[2].id[k];
    pm = pc;
    pc = pc1;
    px = px1;
    py = py1;
    u = u1;
    v = v1;
    w = w1;
    c += plane;
    iu += su;
    iv += sv;
    iw += plane;
  }
}

// Block maxima of |net flux| and |face flux|; non-finite values count as +inf.
__device__ __forceinline__ double fin_abs(double v) {
  const double a = fabs(v);
  return (a <= 1.7976931348623157e308) ? a : __builtin_inf();
}

__global__ void __launch_bounds__(256) div_measure_kernel(Grid g, const double* __restrict__ y,
                                                          double* __restrict__ part) {
  __shared__ double s0[256], s1[256];
  const int t = threadIdx.x;
  double mb = 0.0, mf = 0.0;
  const int64_t C = (int64_t)g.nx * g.ny * g.nz;
  for (int64_t c = (int64_t)blockIdx.x * 256 + t; c < C; c += (int64_t)gridDim.x * 256) {
    const int i = (int)(c % g.nx);
    const int j = (int)((c / g.nx) % g.ny);
    const int k = (int)(c / ((int64_t)g.nx * g.ny));
    const double hx = g.ax[0].h[i], hy = g.ax[1].h[j], hz = g.ax[2].h[k];
    const double u0 = Uat(y, g, i, j, k), u1 = Uat(y, g, i + 1, j, k);
    const double v0 = Vat(y, g, i, j, k), v1 = Vat(y, g, i, j + 1, k);
    const double w0 = Wat(y, g, i, j, k), w1 = Wat(y, g, i, j, k + 1);
    const double net = hy * hz * (u1 - u0) + hx * hz * (v1 - v0) + hx * hy * (w1 - w0);
    mb = fmax(mb, fin_abs(net));
    mf = fmax(mf, fmax(fin_abs(u0 * hy * hz), fmax(fin_abs(v0 * hx * hz), fin_abs(w0 * hx * hy))));
  }
  s0[t] = mb;
  s1[t] = mf;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s0[t] = fmax(s0[t], s0[t + o]);
      s1[t] = fmax(s1[t], s1[t + o]);
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

// Block maxima of the three symmetry measures over theta = T - (1/2 - x_c)
// (T is the centred temperature), Eqs. 7-9.
__global__ void __launch_bounds__(256) symmetry_kernel(Grid g, const double* __restrict__ X, const double* __restrict__ cx,
                                                       double* __restrict__ part) {
  __shared__ double s[3][256];
  const int t = threadIdx.x;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t C = (int64_t)nx * ny * nz;
  for (int64_t c = (int64_t)blockIdx.x * 256 + t; c < C; c += (int64_t)gridDim.x * 256) {
    const int i = (int)(c % nx);
    const int j = (int)((c / nx) % ny);
    const int k = (int)(c / ((int64_t)nx * ny));
    const int im = nx - 1 - i, jm = ny - 1 - j, km = nz - 1 - k;
    const double th = Tat(X, g, i, j, k) - (0.5 - cx[i]);
    const double th_ref = Tat(X, g, i, jm, k) - (0.5 - cx[i]);
    const double th_2d = Tat(X, g, im, j, km) - (0.5 - cx[im]);
    const double th_3d = Tat(X, g, im, jm, km) - (0.5 - cx[im]);
    r0 = fmax(r0, fin_abs(th - th_ref));
    r1 = fmax(r1, fin_abs(th + th_2d));
    r2 = fmax(r2, fin_abs(th + th_3d));
  }
  s[0][t] = r0;
  s[1][t] = r1;
  s[2][t] = r2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o)
      for (int q = 0; q < 3; ++q) s[q][t] = fmax(s[q][t], s[q][t + o]);
    __syncthreads();
  }
  if (t == 0)
    for (int q = 0; q < 3; ++q) part[3 * blockIdx.x + q] = s[q][0];
}

// Projection onto a symmetry class of perturbations (Sec. 2, Eqs. 7-9), one
// packed field of extents (ex, ey, ez), x fastest.  R mirrors y, O mirrors x
// and z; on a mirror-symmetric grid a mirrored face or cell is the reversed
// index.  cr, co: the class sign times the field's sign under R, O (0 for a
// map that is not restricted).  One thread owns the orbit {p, Rp, Op, ROp},
// reads all of it before writing it, and no two threads share an orbit, so
// y may equal x.  Points fixed by a map (middle rows) come out as the
// definition gives: zero where the class is odd there.
__global__ void __launch_bounds__(256) symmetry_class_kernel(const double* x, double* y, int ex, int ey, int ez,
                                                             double cr, double co) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  const int im = ex - 1 - i, jm = ey - 1 - j, km = ez - 1 - k;
  if (i >= ex || j > jm || k > km || (k == km && i > im)) return;
  const int64_t pp = ((int64_t)k * ey + j) * ex + i;
  const int64_t pr = ((int64_t)k * ey + jm) * ex + i;
  const int64_t po = ((int64_t)km * ey + j) * ex + im;
  const int64_t pro = ((int64_t)km * ey + jm) * ex + im;
  double a = x[pp], b = x[pr], c = x[po], d = x[pro];
  if (cr != 0.0) {
    a = 0.5 * (a + cr * b);
    b = cr * a;
    c = 0.5 * (c + cr * d);
    d = cr * c;
  }
  if (co != 0.0) {
    a = 0.5 * (a + co * c);
    c = co * a;
    b = 0.5 * (b + co * d);
    d = co * b;
  }
  y[pp] = a;
  y[pr] = b;
  y[po] = c;
  y[pro] = d;
}

__global__ void max_finish_kernel(const double* __restrict__ part, int nblk, int nq, double* __restrict__ out) {
  __shared__ double s[256];
  const int t = threadIdx.x;
  for (int q = 0; q < nq; ++q) {
    double m = 0.0;
    for (int b = t; b < nblk; b += 256) m = fmax(m, part[nq * b + q]);
    s[t] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) s[t] = fmax(s[t], s[t + o]);
      __syncthreads();
    }
    if (t == 0) out[q] = s[0];
    __syncthreads();
  }
}

inline dim3 cell_block(const Grid& g) { return dim3(64, 4, 1); }
inline dim3 cell_grid(const Grid& g) { return dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz); }
// 16 planes per block, fewer until about 1024 blocks exist
inline dim3 march_grid(const Grid& g) {
  const int64_t tiles = (int64_t)((g.nx + 63) / 64) * ((g.ny + 3) / 4);
  int kd = 16;
  while (kd > 1 && tiles * ((g.nz + kd - 1) / kd) < 1024) kd /= 2;
  return dim3((g.nx + 63) / 64, (g.ny + 3) / 4, (g.nz + kd - 1) / kd);
}

}  // namespace

namespace {

// Launch shape of the tiled stencil: tiles, z-chunk and (padded) block count.
struct TiledShape {
  int tx, ty, kc, ch;
  unsigned blocks;
};

TiledShape tiled_shape(const Grid& g) {
  TiledShape t;
  // z-chunk: 32 planes, shortened on small grids until about 1024 blocks
  // exist (four per CU; one block is 4 waves), but not below 4 planes, since
  // every chunk also loads the plane below and the two above it
  t.tx = (g.nx + TX - 1) / TX;
  t.ty = (g.ny + TY - 1) / TY;
  t.kc = 32;
  while (t.kc > 4 && (int64_t)t.tx * t.ty * ((g.nz + t.kc - 1) / t.kc) < 1024) t.kc /= 2;
  t.ch = (g.nz + t.kc - 1) / t.kc;
  const int64_t total = (int64_t)t.tx * t.ty * t.ch;
  t.blocks = (unsigned)(((total + 7) / 8) * 8);
  return t;
}

// LDS per block: 14 planes for J, 7 for N, plus for the fused divergence
// the u, v, w faces of the tile, each thread's carried flux and the
// columns' sqrt(h_x) (51.8 KB: three blocks still share a CU's 160 KB)
constexpr size_t kLdsJ = 14 * PLANE * sizeof(double), kLdsN = 7 * PLANE * sizeof(double);
constexpr size_t kLdsJDiv = kLdsJ + (4 * TX * TY + TX) * sizeof(double);

// raise the dynamic-LDS limit of a kernel explicitly, whatever its default
// (once per kernel and process; the static's initialization is thread-safe)
template <const void* (*K)()>
bool tiled_lds_ok(size_t bytes) {
  static const bool ok =
      hipFuncSetAttribute(K(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
  return ok;
}
const void* kernel_j() { return reinterpret_cast<const void*>(&operator_tiled_kernel<0>); }
const void* kernel_jdiv() { return reinterpret_cast<const void*>(&operator_divergence_kernel); }

// the tiled kernels address a vector with 32-bit byte offsets
bool tiled_fits(const Grid& g) { return g.n * 8 < ((int64_t)1 << 31); }

}  // namespace

hipError_t launch_operator(const kv_ctx* c, const double* X0, const double* x, double* y, int mode) {
  const Grid& g = c->g;
  if (!tiled_fits(g) || (mode == 0 && !tiled_lds_ok<kernel_j>(kLdsJ))) {
    // the one-cell-per-thread kernel
    if (mode == 0)
      operator_kernel<0><<<cell_grid(g), cell_block(g), 0, c->stream>>>(g, X0, x, y);
    else
      operator_kernel<1><<<cell_grid(g), cell_block(g), 0, c->stream>>>(g, x, x, y);
    return hipGetLastError();
  }
  const TiledShape t = tiled_shape(g);
  if (mode == 0)
    operator_tiled_kernel<0><<<t.blocks, 256, kLdsJ, c->stream>>>(g, X0, x, y, t.tx, t.ty, t.ch, t.kc);
  else
    operator_tiled_kernel<1><<<t.blocks, 256, kLdsN, c->stream>>>(g, x, x, y, t.tx, t.ty, t.ch, t.kc);
  return hipGetLastError();
}

bool operator_fuses_divergence(const kv_ctx* c) {
  return tiled_fits(c->g) && tiled_lds_ok<kernel_jdiv>(kLdsJDiv);
}

hipError_t launch_operator_divergence(const kv_ctx* c, const double* X0, const double* x, double* y,
                                      double* div) {
  const Grid& g = c->g;
  if (!operator_fuses_divergence(c)) return hipErrorNotSupported;
  const TiledShape t = tiled_shape(g);
  operator_divergence_kernel<<<t.blocks, 256, kLdsJDiv, c->stream>>>(g, X0, x, y, t.tx, t.ty, t.ch, t.kc, div);
  return hipGetLastError();
}

hipError_t launch_divergence_edges(const kv_ctx* c, const double* y, double* div) {
  const Grid& g = c->g;
  const int kc = tiled_shape(g).kc;
  const int cx = (g.nx - 1) / TX, cy = (g.ny - 1) / TY, cz = (g.nz - 1) / kc;
  const int64_t nbx = (g.nx + 255) / 256, nby = (g.ny + 255) / 256;
  const int64_t b1 = nbx * cy * ((g.nz + EDGE_KQ - 1) / EDGE_KQ), b2 = (int64_t)cx * nby * g.nz,
                b3 = nbx * g.ny * cz;
  const int64_t blocks = b1 + b2 + b3;
  if (blocks == 0) return hipSuccess;
  if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  divergence_edges_kernel<<<(unsigned)blocks, 256, 0, c->stream>>>(g, y, div, kc, cx, cy, (unsigned)b1,
                                                                   (unsigned)b2);
  return hipGetLastError();
}

hipError_t launch_scaled_divergence(const kv_ctx* c, const double* y, double* out) {
  const Grid& g = c->g;
  scaled_divergence_kernel<double><<<march_grid(g), cell_block(g), 0, c->stream>>>(g, y, out);
  return hipGetLastError();
}

hipError_t launch_scaled_divergence_f32(const kv_ctx* c, const double* y, float* out) {
  const Grid& g = c->g;
  scaled_divergence_kernel<float><<<march_grid(g), cell_block(g), 0, c->stream>>>(g, y, out);
  return hipGetLastError();
}

hipError_t launch_correct_divergence(kv_ctx* c, const double* yin, const float* p, double* yout, float* bnext) {
  const Grid& g = c->g;
  const dim3 grid = march_grid(g);
  const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
  if (2 * nblk > c->cell_part_len) return hipErrorInvalidValue;
  correct_divergence_kernel<<<grid, cell_block(g), 0, c->stream>>>(g, yin, p, yout, bnext, c->cell_part);
  max_finish_kernel<<<1, 256, 0, c->stream>>>(c->cell_part, (int)nblk, 2, c->dres);
  return hipGetLastError();
}

hipError_t launch_gradient_correction(const kv_ctx* c, const double* p, double* y) {
  const Grid& g = c->g;
  gradient_correction_kernel<<<march_grid(g), cell_block(g), 0, c->stream>>>(g, p, y);
  return hipGetLastError();
}

hipError_t launch_div_measure(kv_ctx* c, const double* y) {
  const int nblk = c->npart_blocks;
  div_measure_kernel<<<nblk, 256, 0, c->stream>>>(c->g, y, c->part);
  max_finish_kernel<<<1, 256, 0, c->stream>>>(c->part, nblk, 2, c->dres);
  return hipGetLastError();
}

hipError_t launch_symmetry(kv_ctx* c, const double* X) {
  const int nblk = c->npart_blocks;
  symmetry_kernel<<<nblk, 256, 0, c->stream>>>(c->g, X, c->g.ax[0].c, c->part);
  max_finish_kernel<<<1, 256, 0, c->stream>>>(c->part, nblk, 3, c->dres);
  return hipGetLastError();
}

hipError_t launch_symmetry_class(kv_ctx* c, const double* x, double* y, int e_ref, int e_rot) {
  const Grid& g = c->g;
  const int ext[4][3] = {{g.nx - 1, g.ny, g.nz}, {g.nx, g.ny - 1, g.nz}, {g.nx, g.ny, g.nz - 1}, {g.nx, g.ny, g.nz}};
  const int64_t off[4] = {g.ou, g.ov, g.ow, g.oT};
  // field signs under the reflection y -> 1-y and the rotation (x,z) -> (1-x,1-z)
  const double s_ref[4] = {1.0, -1.0, 1.0, 1.0};
  const double s_rot[4] = {-1.0, 1.0, -1.0, -1.0};
  for (int f = 0; f < 4; ++f) {
    const int ex = ext[f][0], ey = ext[f][1], ez = ext[f][2];
    if (ex <= 0 || ey <= 0 || ez <= 0) continue;
    const dim3 grid((ex + 63) / 64, ((ey + 1) / 2 + 3) / 4, (ez + 1) / 2);
    symmetry_class_kernel<<<grid, dim3(64, 4, 1), 0, c->stream>>>(x + off[f], y + off[f], ex, ey, ez,
                                                                   e_ref * s_ref[f], e_rot * s_rot[f]);
  }
  return hipGetLastError();
}

}  // namespace kv
