// C ABI of the Krylov-vector library: context, base flow, the projected
// Jacobian, the residual, and the Newton (BiCGstab(2) + GMRES) and
// Chebyshev-Arnoldi drivers.  The drivers run on the host and launch the
// device kernels; only small scalars (dot products, the Hessenberg matrix,
// Ritz data) cross to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kv_internal.h"

namespace kv {
hipError_t launch_hessenberg_values(hipStream_t s, double* Hwork, int m, double* wr, double* wi, int* info);
hipError_t launch_hessenberg_vectors(hipStream_t s, const double* H, int m, const double* lr, const double* li,
                                     int nsel, double* cwork, double* vr, double* vi);
}  // namespace kv

using namespace kv;

namespace {

const char* kNoCtx = "kv: null context";

int fail(kv_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(c, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail((c), KV_EDEVICE, std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call); \
  } while (0)

// ---- host metrics -----------------------------------------------------------------
struct HostAxis {
  int n;
  std::vector<double> h, ih, id, wlo, whi, sq, isq, dd, lam, c, Q, Qt;
  int null_idx;
  bool split = false;  // Q / Qt hold the even/odd half bases [2][H][H]
};

void general_basis(HostAxis& a, std::vector<double>& M);

bool build_axis(const double* f, int n, HostAxis& a, std::string& err, bool allow_split = true) {
  a.n = n;
  if (std::fabs(f[0]) > 1e-14 || std::fabs(f[n] - 1.0) > 1e-14) {
    err = "faces must start at 0 and end at 1";
    return false;
  }
  for (int i = 0; i < n; ++i)
    if (!(f[i + 1] > f[i])) {
      err = "faces must be strictly increasing";
      return false;
    }
  a.h.resize(n);
  a.ih.resize(n);
  a.sq.resize(n);
  a.isq.resize(n);
  a.c.resize(n);
  a.id.assign(n + 1, 0.0);
  a.dd.assign(n + 1, 0.0);
  a.wlo.assign(n + 1, 0.0);
  a.whi.assign(n + 1, 0.0);
  for (int i = 0; i < n; ++i) {
    a.h[i] = f[i + 1] - f[i];
    a.ih[i] = 1.0 / a.h[i];
    a.c[i] = 0.5 * (f[i] + f[i + 1]);
    a.sq[i] = std::sqrt(a.h[i]);
    a.isq[i] = 1.0 / a.sq[i];
  }
  a.dd[0] = 0.5 * a.h[0];
  a.dd[n] = 0.5 * a.h[n - 1];
  // midpoint centres: the centre gap is (h_{i-1} + h_i)/2 and the weights of
  // cells i-1 and i at face i are (h_i/2)/d_i and (h_{i-1}/2)/d_i
  for (int i = 1; i < n; ++i) {
    a.dd[i] = 0.5 * (a.h[i - 1] + a.h[i]);
    a.wlo[i] = (0.5 * a.h[i]) / a.dd[i];
    a.whi[i] = (0.5 * a.h[i - 1]) / a.dd[i];
  }
  for (int i = 0; i <= n; ++i) a.id[i] = 1.0 / a.dd[i];
  // M = H^-1/2 K H^-1/2, K the symmetric tridiagonal Neumann operator
  std::vector<double> M((size_t)n * n, 0.0);
  for (int i = 0; i + 1 < n; ++i) {
    const double t = a.id[i + 1];
    M[(size_t)i * n + i + 1] += t * a.isq[i] * a.isq[i + 1];
    M[(size_t)(i + 1) * n + i] += t * a.isq[i] * a.isq[i + 1];
    M[(size_t)i * n + i] -= t * a.isq[i] * a.isq[i];
    M[(size_t)(i + 1) * n + i + 1] -= t * a.isq[i + 1] * a.isq[i + 1];
  }
  // Mirror-symmetric axis (h_i = h_{n-1-i} to round-off, n even): M is
  // persymmetric and its eigenvectors are [w; +-J w]/sqrt(2) with w the
  // eigenvectors of the half blocks M_11 +- M_{H-1,H} e_{H-1} e_{H-1}^T.
  bool sym = allow_split && (n % 2 == 0) && n >= 4;
  for (int i = 0; sym && i < n; ++i)
    if (a.h[i] != a.h[n - 1 - i]) sym = false;
  if (sym) {
    const int H = n / 2;
    std::vector<double> Ms((size_t)n * n);
    for (int r = 0; r < n; ++r)
      for (int cc = 0; cc < n; ++cc)
        Ms[(size_t)r * n + cc] = 0.5 * (M[(size_t)r * n + cc] + M[(size_t)(n - 1 - r) * n + (n - 1 - cc)]);
    const double t = Ms[(size_t)(H - 1) * n + H];
    std::vector<double> Wp[2], lp[2];
    for (int par = 0; par < 2; ++par) {
      std::vector<double> Mh((size_t)H * H);
      for (int r = 0; r < H; ++r)
        for (int cc = 0; cc < H; ++cc) Mh[(size_t)r * H + cc] = Ms[(size_t)r * n + cc];
      Mh[(size_t)(H - 1) * H + (H - 1)] += par ? -t : t;
      jacobi_eigen(H, Mh, Wp[par], lp[par]);
    }
    a.split = true;
    a.lam.resize(n);
    a.Q.assign((size_t)2 * H * H, 0.0);
    a.Qt.assign((size_t)2 * H * H, 0.0);
    const double rs2 = 1.0 / std::sqrt(2.0);
    for (int par = 0; par < 2; ++par)
      for (int e = 0; e < H; ++e) {
        a.lam[par * H + e] = lp[par][e];
        for (int k = 0; k < H; ++k) {
          const double q = Wp[par][(size_t)k * H + e] * rs2;
          a.Q[(size_t)par * H * H + (size_t)k * H + e] = q;
          a.Qt[(size_t)par * H * H + (size_t)e * H + k] = q;
        }
      }
    // the constant mode is symmetric: the largest even eigenvalue
    a.null_idx = (int)(std::max_element(a.lam.begin(), a.lam.begin() + H) - a.lam.begin());
    a.lam[a.null_idx] = 0.0;  // K annihilates constants: the exact eigenvalue is 0
    return true;
  }
  general_basis(a, M);
  return true;
}

// Full n x n eigenbasis of M (no even/odd split).
void general_basis(HostAxis& a, std::vector<double>& M) {
  const int n = a.n;
  a.split = false;
  jacobi_eigen(n, M, a.Q, a.lam);
  a.null_idx = (int)(std::max_element(a.lam.begin(), a.lam.end()) - a.lam.begin());
  a.lam[a.null_idx] = 0.0;  // K annihilates constants: the exact eigenvalue is 0
  a.Qt.resize((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int cc = 0; cc < n; ++cc) a.Qt[(size_t)cc * n + r] = a.Q[(size_t)r * n + cc];
}

void build_axis_general(const double* f, int n, HostAxis& a) {
  std::string err;
  build_axis(f, n, a, err, false);
}

// ---- small device helpers -----------------------------------------------------------
int read_results(kv_ctx* c, int nq) {
  HIPCHK(c, hipMemcpyAsync(c->hres, c->dres, sizeof(double) * nq, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return KV_OK;
}

// Host -> device copy that completes before returning (the host buffer may be
// a temporary).
int upload(kv_ctx* c, void* dst, const void* src, size_t bytes) {
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return KV_OK;
}

int dots(kv_ctx* c, int np, const double* const* a, const double* const* b, double* out) {
  HIPCHK(c, launch_wdots(c, np, a, b));
  int rc = read_results(c, np);
  if (rc) return rc;
  for (int q = 0; q < np; ++q) out[q] = c->hres[q];
  return KV_OK;
}

double dot1(kv_ctx* c, const double* a, const double* b, int* rc) {
  double v = 0;
  *rc = dots(c, 1, &a, &b, &v);
  return v;
}

int lincomb(kv_ctx* c, int nt, std::initializer_list<double> cf, std::initializer_list<const double*> in,
            double* out) {
  std::vector<double> cc(cf);
  std::vector<const double*> pp(in);
  HIPCHK(c, launch_lincomb(c, c->g.n, nt, cc.data(), pp.data(), out));
  return KV_OK;
}

// Phase timing: an event pair around a phase while kv_timing is enabled.
hipEvent_t take_event(kv_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct PhaseMark {
  kv_ctx* c;
  int phase;
  hipEvent_t e0 = nullptr;
  PhaseMark(kv_ctx* cc, int ph) : c(cc), phase(ph) {
    if (c->timing && (e0 = take_event(c))) hipEventRecord(e0, c->stream);
  }
  ~PhaseMark() {
    if (!e0) return;
    hipEvent_t e1 = take_event(c);
    if (!e1) return;
    hipEventRecord(e1, c->stream);
    c->ev_marks.push_back({phase, {e0, e1}});
  }
};

// The FP64 projection from the scaled divergence of y already in cellA.
int project_from_divergence(kv_ctx* c, double* y) {
  {
    PhaseMark pm(c, 2);
    HIPCHK(c, launch_fd_solve(c, c->cellA, c->cellA));
  }
  {
    PhaseMark pm(c, 3);
    HIPCHK(c, launch_gradient_correction(c, c->cellA, y));
  }
  return KV_OK;
}

int project_inplace(kv_ctx* c, double* y) {
  if (c->solve_mixed) return kv::project_mixed_with(c, y, nullptr, nullptr, c->ymix_solve);
  {
    PhaseMark pm(c, 1);
    HIPCHK(c, launch_scaled_divergence(c, y, c->cellA));
  }
  return project_from_divergence(c, y);
}

// Mixed form of the projection: FP32-storage fast diagonalization on the
// FP32 matrix cores, refined on the FP64 residual.  Each sweep solves for
// the divergence left by the previous one; corrections and the next
// divergence are fused, and the sweeps alternate between y and a scratch
// vector (an odd count ends with
// a copy of the velocity back into y).  Stops when the normalized divergence
// max|net flux| / max|face flux| <= tol, checked from the second sweep on (at
// most 8 sweeps).
constexpr double kMixedDivTol = 1e-10;

// Transforms of the mixed sweeps: FP32 products on the FP32 matrix cores
// (default), or KV_MIXED_FD=bf16x3 for bf16x3 split products on the bf16
// matrix cores (read at every call, for tests and measurements).  The bf16x3
// passes are more accurate per sweep but, with their operands split and
// transposed in LDS, slower than the FP32 ones on this hardware.
bool mixed_fd_bf16x3() {
  const char* e = getenv("KV_MIXED_FD");
  return e && std::strcmp(e, "bf16x3") == 0;
}

int ws_bind(kv_ctx* c, int op, int m, int neig);

}  // namespace

// The mixed projection with its scratch vector ymix (n doubles, any device
// memory the caller provides: the workspace, or the library's static scratch
// for kv_project_mixed_static).
int kv::project_mixed_with(kv_ctx* c, double* y, double* div_out, int* sweeps_out, double* ymix) {
  const int64_t C = c->ncell;
  int rc;
  // FP32 fields inside the two FP64 cell buffers
  float* F0 = reinterpret_cast<float*>(c->cellA);
  float* F1 = F0 + C;
  {
    PhaseMark pm(c, 1);
    HIPCHK(c, launch_scaled_divergence_f32(c, y, F0));
  }
  double div = 1.0;
  int sweeps = 0;
  while (sweeps < 8) {
    // even sweeps read y and write the scratch vector, odd ones the reverse
    const bool from_y = sweeps % 2 == 0;
    const double* src = from_y ? y : ymix;
    double* dst = from_y ? ymix : y;
    float* b = from_y ? F0 : F1;
    float* bn = from_y ? F1 : F0;
    {
      PhaseMark pm(c, 2);
      if (mixed_fd_bf16x3()) HIPCHK(c, launch_fd_solve_bf3(c, b, b));
      else HIPCHK(c, launch_fd_solve_f32(c, b, b));
    }
    {
      PhaseMark pm(c, 3);
      HIPCHK(c, launch_correct_divergence(c, src, b, dst, bn));
    }
    ++sweeps;
    if (sweeps < 2) continue;  // one FP32 sweep never reaches the tolerance
    if ((rc = read_results(c, 2))) return rc;
    div = c->hres[1] > 0 ? c->hres[0] / c->hres[1] : 0.0;
    if (!std::isfinite(div)) return fail(c, KV_ENONFINITE, "non-finite value in the mixed projection");
    if (div <= kMixedDivTol) break;
  }
  if (sweeps % 2 == 1) {
    // the result is in the scratch vector: its velocity back into y (T of y is final)
    PhaseMark pm(c, 3);
    HIPCHK(c, hipMemcpyAsync(y, ymix, c->g.oT * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
  if (div_out) *div_out = div;
  if (sweeps_out) *sweeps_out = sweeps;
  if (div > kMixedDivTol) return fail(c, KV_ENOCONV, "mixed projection: divergence not reduced to 1e-10");
  return KV_OK;
}

bool kv::mixed_grid(const kv_ctx* c) { return c->split[0] && c->split[1] && c->split[2]; }

size_t kv::mixed_scratch_bytes(const kv_ctx* c) { return (size_t)c->g.n * sizeof(double); }

namespace {

int project_mixed(kv_ctx* c, double* y, double* div_out, int* sweeps_out) {
  int rc = ws_bind(c, KV_WS_PROJECT_MIXED, 0, 0);
  if (rc) return rc;
  return project_mixed_with(c, y, div_out, sweeps_out, c->ymix);
}

bool mixed_ok(const kv_ctx* c) { return mixed_grid(c); }

int apply_operator(kv_ctx* c, const double* x, double* y) {
  PhaseMark pm(c, 0);
  HIPCHK(c, launch_operator(c, c->X0, x, y, 0));
  return KV_OK;
}

// The stencil writes the scaled divergence of its output itself unless
// KV_FUSED_DIV=0 (read at every call, for tests and measurements), where
// the separate divergence pass runs.
bool fused_divergence_on(const kv_ctx* c) {
  const char* e = getenv("KV_FUSED_DIV");
  return !(e && std::strcmp(e, "0") == 0) && operator_fuses_divergence(c);
}

// y = P J(X0) x in FP64 (the mixed projection when the solvers use it)
int apply_projected(kv_ctx* c, const double* x, double* y) {
  if (c->solve_mixed || !fused_divergence_on(c)) {
    int rc = apply_operator(c, x, y);
    if (rc) return rc;
    return project_inplace(c, y);
  }
  {
    PhaseMark pm(c, 0);
    HIPCHK(c, launch_operator_divergence(c, c->X0, x, y, c->cellA));
  }
  {
    PhaseMark pm(c, 1);
    HIPCHK(c, launch_divergence_edges(c, y, c->cellA));
  }
  return project_from_divergence(c, y);
}

// y <- (I - Q Q^T W) y over the locked vectors Q (classical Gram-Schmidt
// twice, no host synchronization); nothing while none are locked.
int deflate(kv_ctx* c, double* y) {
  for (int pass = 0; c->nlock > 0 && pass < 2; ++pass) {
    HIPCHK(c, launch_mdot(c, c->lockQ, c->g.n, c->nlock, y));
    HIPCHK(c, launch_mupdate(c, c->lockQ, c->g.n, c->nlock, c->dres, y));
  }
  return KV_OK;
}

int matvec(kv_ctx* c, const double* x, double* y) {
  int rc = apply_projected(c, x, y);
  if (rc) return rc;
  if (c->sym_ref || c->sym_rot) HIPCHK(c, launch_symmetry_class(c, y, y, c->sym_ref, c->sym_rot));
  return deflate(c, y);
}

// Class signs (+1 symmetric, -1 antisymmetric, 0 free) from KV_SYM_* bits;
// false on an unknown bit or both signs of one map.
bool sym_class(unsigned sym, int* e_ref, int* e_rot) {
  const unsigned all = KV_SYM_REF_EVEN | KV_SYM_REF_ODD | KV_SYM_ROT_EVEN | KV_SYM_ROT_ODD;
  if (sym & ~all) return false;
  if ((sym & KV_SYM_REF_EVEN) && (sym & KV_SYM_REF_ODD)) return false;
  if ((sym & KV_SYM_ROT_EVEN) && (sym & KV_SYM_ROT_ODD)) return false;
  *e_ref = (sym & KV_SYM_REF_EVEN) ? 1 : (sym & KV_SYM_REF_ODD) ? -1 : 0;
  *e_rot = (sym & KV_SYM_ROT_EVEN) ? 1 : (sym & KV_SYM_ROT_ODD) ? -1 : 0;
  return true;
}

// Widths mirror-symmetric about the axis midpoint (to 1e-12 of the largest).
bool mirror_axis(const kv_ctx* c, int a) {
  const std::vector<double>& f = c->hf[a];
  const int n = (int)f.size() - 1;
  double hmax = 0.0;
  for (int i = 0; i < n; ++i) hmax = std::max(hmax, f[i + 1] - f[i]);
  for (int i = 0; i < n; ++i)
    if (std::fabs((f[i + 1] - f[i]) - (f[n - i] - f[n - 1 - i])) > 1e-12 * hmax) return false;
  return true;
}

int check_sym(kv_ctx* c, unsigned sym, int* e_ref, int* e_rot) {
  if (!sym_class(sym, e_ref, e_rot)) return fail(c, KV_EINVAL, "bad symmetry-class flags");
  if ((*e_ref && !mirror_axis(c, 1)) || (*e_rot && !(mirror_axis(c, 0) && mirror_axis(c, 2))))
    return fail(c, KV_EINVAL, "symmetry class needs a grid mirror-symmetric along the mirrored axes");
  return KV_OK;
}

// Keeps matvec in a symmetry class and deflated by the locked vectors for
// one eigen-solve, cleared on every exit.
struct EigScope {
  kv_ctx* c;
  EigScope(kv_ctx* cc, int er, int eo, const double* Q) : c(cc) {
    c->sym_ref = er;
    c->sym_rot = eo;
    c->lockQ = Q;
    c->nlock = 0;
  }
  ~EigScope() {
    c->sym_ref = c->sym_rot = 0;
    c->lockQ = nullptr;
    c->nlock = 0;
  }
};

// Makes every projection of one solver call the mixed form when the
// context asks for it (kv_set_solver_projection); cleared on every exit.
struct MixedScope {
  kv_ctx* c;
  explicit MixedScope(kv_ctx* cc) : c(cc) { c->solve_mixed = c->solve_mixed_set; }
  ~MixedScope() { c->solve_mixed = false; }
};

// y = M^-1 x of the Stokes/heat preconditioner: per block the Helmholtz
// solve (sigma - nu Lap_v) or (sigma - kappa Lap_T), then P on the velocity.
int precond_apply(kv_ctx* c, const double* x, double* y) {
  const Grid& g = c->g;
  const int64_t off[4] = {g.ou, g.ov, g.ow, g.oT};
  const HelmBasis *bx[4], *by[4], *bz[4];
  double coef[4];
  const double* in[4];
  double *out[4], *scr[4];
  for (int b = 0; b < 4; ++b) {
    bx[b] = &c->hb[0][b == 3 ? HB_CD : (b == 0 ? HB_FD : HB_CD)];
    by[b] = &c->hb[1][b == 3 ? HB_CN : (b == 1 ? HB_FD : HB_CD)];
    bz[b] = &c->hb[2][b == 3 ? HB_CN : (b == 2 ? HB_FD : HB_CD)];
    coef[b] = b == 3 ? g.kappa : g.nu;
    in[b] = x + off[b];
    out[b] = y + off[b];
    scr[b] = c->pc_scr + off[b];
  }
  HIPCHK(c, launch_fd_helmholtz4(c, bx, by, bz, c->pc_sigma, coef, in, out, scr));
  return project_inplace(c, y);
}

int cayley_apply(kv_ctx* c, const double* x, double* y);

// The operator of the Krylov solvers: P J, or P J M^-1 while a
// preconditioned Newton correction runs.  While a transformed Arnoldi runs
// it is the Cayley operator (cayley_apply), and inside that operator's
// inner solve (P J - pole) M^-1.
int op_apply(kv_ctx* c, const double* x, double* y) {
  if (c->st_on && !c->st_inner) return cayley_apply(c, x, y);
  const double* u = x;
  int rc;
  if (c->pc_active) {
    if ((rc = precond_apply(c, x, c->pc_tmp))) return rc;
    u = c->pc_tmp;
  }
  if ((rc = matvec(c, u, y))) return rc;
  if (c->st_inner) return lincomb(c, 2, {1.0, -c->st_pole}, {y, u}, y);
  return KV_OK;
}

int check_finite(kv_ctx* c, const double* a, int64_t n, const char* what) {
  HIPCHK(c, launch_maxabs(c, a, n));
  int rc = read_results(c, 1);
  if (rc) return rc;
  if (!std::isfinite(c->hres[0])) return fail(c, KV_ENONFINITE, std::string("non-finite value in ") + what);
  return KV_OK;
}

// ---- caller workspace ------------------------------------------------------------------
// Doubles of the Hessenberg / Ritz-vector area for k Arnoldi steps and nsel
// wanted values: H_k and a copy, eigenvalues, selected values, coefficient
// vectors, info, and a k x k complex matrix plus a right-hand side per value.
size_t hess_area(int k, int nsel) {
  const size_t kk = (size_t)k * k;
  return 4 * kk + 4 * (size_t)k + 2 + 2 * (size_t)nsel * (kk + (size_t)k);
}

// Vectors of a spectral transform's inner solve: its iterate, the GMRES
// basis and, with a preconditioner, M^-1 x and the Helmholtz scratch.
size_t st_vectors(const kv_ctx* c) {
  if (c->st_kind == KV_ST_NONE) return 0;
  return 1 + (size_t)c->gmres_m + 1 + (c->pc_kind != KV_PC_NONE ? 2 : 0);
}

// Packed vectors an operation carves from the workspace (see ws_bind).
size_t ws_vectors(const kv_ctx* c, int op, int m, int neig) {
  switch (op) {
    case KV_WS_PROJECT_MIXED: return 1;
    case KV_WS_APPLY_PRECONDITIONER: return 1;
    case KV_WS_NEWTON:
      return 8 + (size_t)c->gmres_m + 1 + (c->pc_kind != KV_PC_NONE ? 3 : 0) + (c->gmres_defl ? 1 : 0) +
             (c->solve_mixed_set ? 1 : 0);
    case KV_WS_ARNOLDI: return (size_t)m + 4 + 2 * (size_t)(neig + 1) + st_vectors(c) + (c->solve_mixed_set ? 1 : 0);
    case KV_WS_TIME_STEPS: return 4;
    default: return 0;
  }
}

// Ritz vectors the Hessenberg area holds: the wanted set (n_eigs + 1 with a
// pair kept whole), or a thick restart's kept set (at most 64)
int ritz_slots(int m, int neig) { return std::max(neig + 1, std::min(m, 64)); }

size_t ws_need(const kv_ctx* c, int op, int m, int neig) {
  size_t bytes = ws_vectors(c, op, m, neig) * (size_t)c->g.n * sizeof(double);
  if (op == KV_WS_ARNOLDI) bytes += hess_area(m, ritz_slots(m, neig)) * sizeof(double);
  if (op == KV_WS_NEWTON && c->gmres_defl) bytes += hess_area(c->gmres_m, c->gmres_defl + 1) * sizeof(double);
  return bytes;
}

// Points the per-call scratch of an operation into the caller's workspace
// (KV_EINVAL when none is set or it is too small).  Layouts, in packed
// vectors of n doubles:
//   PROJECT_MIXED          ymix
//   APPLY_PRECONDITIONER   pc_scr
//   NEWTON                 8 BiCGstab(2) vectors | GMRES basis (m+1) | pc_tmp pc_d0 pc_scr |
//                          (mixed solver projection) ymix_solve |
//                          (deflated GMRES) a spare vector, the Hessenberg area
//   ARNOLDI                V (m+1) | zp zc tmp | locked (neig+1) | Ritz (neig+1) |
//                          (spectral transform) inner iterate, GMRES basis (gmres_m+1),
//                          (with a preconditioner) pc_tmp pc_scr | (mixed solver
//                          projection) ymix_solve | Hessenberg area
//   TIME_STEPS             F | F of the previous step | right-hand side | pc_scr
int ws_bind(kv_ctx* c, int op, int m, int neig) {
  const size_t need = ws_need(c, op, m, neig);
  if (!c->ws || c->ws_bytes < need) {
    char msg[160];
    snprintf(msg, sizeof msg, "workspace too small: the call needs %zu bytes, %zu are set (kv_workspace_size, kv_set_workspace)",
             need, c->ws ? c->ws_bytes : (size_t)0);
    return fail(c, KV_EINVAL, msg);
  }
  const int64_t n = c->g.n;
  switch (op) {
    case KV_WS_PROJECT_MIXED: c->ymix = c->ws; break;
    case KV_WS_APPLY_PRECONDITIONER: c->pc_scr = c->ws; break;
    case KV_WS_NEWTON: {
      double* p = c->ws + (int64_t)(8 + c->gmres_m + 1) * n;
      if (c->pc_kind != KV_PC_NONE) {
        c->pc_tmp = p;
        c->pc_d0 = p + n;
        c->pc_scr = p + 2 * n;
        p += 3 * n;
      }
      if (c->solve_mixed_set) {
        c->ymix_solve = p;
        p += n;
      }
      if (c->gmres_defl) c->hess = p + n;  // after one spare vector
      break;
    }
    case KV_WS_ARNOLDI: {
      double* p = c->ws + (int64_t)(m + 4 + 2 * (neig + 1)) * n;
      if (c->st_kind != KV_ST_NONE) {
        c->st_t = p;
        c->st_V = p + n;
        p += (int64_t)(c->gmres_m + 2) * n;
        if (c->pc_kind != KV_PC_NONE) {
          c->pc_tmp = p;
          c->pc_scr = p + n;
          p += 2 * n;
        }
      }
      if (c->solve_mixed_set) {
        c->ymix_solve = p;
        p += n;
      }
      c->hess = p;
      break;
    }
    case KV_WS_TIME_STEPS: c->pc_scr = c->ws + 3 * n; break;
    default: return fail(c, KV_EINVAL, "unknown workspace operation");
  }
  return KV_OK;
}

// ---- Arnoldi with delayed classical Gram-Schmidt twice ---------------------------------------
// V holds up to m+1 vectors (stride n).  On entry V[j0] is the next vector
// (W-normalized for j0 = 0) and, for j0 > 0, V[0..j0) and the columns < j0 of H
// (with row j0) come from a thick restart.  Fills H ((m+1) x m, column-major
// by j: H[i + j*(m+1)]) and returns the number of completed steps k (k < m on
// a lucky breakdown); V[0..k] is W-orthonormal on return.
//
// Classical Gram-Schmidt twice with the second pass delayed by one step
// (low-synchronization CGS2): step j applies A to v_j as orthogonalized once,
// then ONE two-vector multi-dot over V[0..j] gives the coefficients that
// finish v_j (s = V^T W v_j, its norm from <v_j, v_j> - |s|^2) and those of
// w = A v_j; the coefficients of A v_j(final) follow on the host from the
// Arnoldi relation already built (A V s = V H s), and ONE fused update pass
// finishes v_j and orthogonalizes w once against V[0..j].  Against plain
// CGS2 this reads the basis twice per step instead of four times and
// synchronizes once.  The last vector gets its second pass at the end.
int arnoldi(kv_ctx* c, double* V, int m, std::vector<double>& H, int* kout, int* matvecs, int j0 = 0) {
  const int64_t n = c->g.n;
  const int ld = m + 1;
  if (j0 == 0) H.assign((size_t)ld * m, 0.0);  // else columns < j0 (and row j0) are kept
  int rc;
  std::vector<double> sv, g, h;
  // finishes v_j (provisional, orthogonalized once) given s = V[0..j)^T W v_j
  // and a = <v_j, v_j>_W: rho and the corrected columns of H; false if v_j
  // vanishes (lucky breakdown)
  auto finish_coeffs = [&](int jj, const double* sj, double a, double* rho_out) -> bool {
    double ss = 0.0;
    for (int i = 0; i < jj; ++i) ss += sj[i] * sj[i];
    const double r2 = a - ss;
    if (!(r2 > 1e-26 * a) || !std::isfinite(r2)) return false;
    const double rho = std::sqrt(r2);
    for (int cc = 0; cc < jj; ++cc) {
      const double hj = H[jj + (size_t)cc * ld];
      if (hj == 0.0) continue;
      for (int i = 0; i < jj; ++i) H[i + (size_t)cc * ld] += hj * sj[i];
      H[jj + (size_t)cc * ld] = hj * rho;
    }
    *rho_out = rho;
    return true;
  };
  for (int j = j0; j < m; ++j) {
    double* vj = V + (int64_t)j * n;
    double* w = V + (int64_t)(j + 1) * n;
    if ((rc = op_apply(c, vj, w))) return rc;
    ++*matvecs;
    HIPCHK(c, launch_mdot2(c, V, n, j + 1, vj, w, c->dres, c->dres + 512));
    if ((rc = read_results(c, 1024))) return rc;
    const double* a = c->hres;        // <V_i, v_j>, i <= j
    const double* b = c->hres + 512;  // <V_i, w>, i <= j
    if (!std::isfinite(a[j]) || !std::isfinite(b[j])) return fail(c, KV_ENONFINITE, "non-finite Arnoldi vector");
    // scale of A v_{j-1} for the breakdown test of v_j
    double col = a[j];
    if (j > 0)
      for (int i = 0; i < j; ++i) col += H[i + (size_t)(j - 1) * ld] * H[i + (size_t)(j - 1) * ld];
    double rho = 0.0;
    sv.assign(a, a + j);
    const bool ok = finish_coeffs(j, sv.data(), a[j], &rho);
    if (!ok || (j > j0 && rho <= 1e-14 * std::sqrt(col))) {
      if (ok) {
        // v_j is tiny: the space is invariant; H[j][j-1] keeps the tiny value
      } else {
        for (int cc = 0; cc < j; ++cc) H[j + (size_t)cc * ld] = 0.0;
      }
      *kout = j;
      if (j == 0) return fail(c, KV_ENONFINITE, "zero Arnoldi start vector");
      return KV_OK;
    }
    // A V s = V H s over the columns < j (H corrected above)
    g.assign(j + 1, 0.0);
    for (int cc = 0; cc < j; ++cc) {
      const double scc = sv[cc];
      if (scc == 0.0) continue;
      for (int i = 0; i <= j; ++i) g[i] += H[i + (size_t)cc * ld] * scc;
    }
    double vw = b[j];
    for (int i = 0; i < j; ++i) vw -= sv[i] * b[i];
    vw /= rho;                                        // <v_j(final), w>
    h.assign(j + 1, 0.0);
    for (int i = 0; i < j; ++i) h[i] = (b[i] - g[i]) / rho;
    h[j] = (vw - g[j]) / rho;
    const double cvj = (g[j] / rho + h[j]) / rho;
    // coefficients of the fused update: w <- w/rho - cvj v_j - V d,
    // v_j <- (v_j - V s)/rho
    double* hc = c->hcoef;
    for (int i = 0; i < j; ++i) {
      hc[i] = g[i] / rho + h[i] - cvj * sv[i];
      hc[512 + i] = sv[i];
    }
    if (j > 0)
      HIPCHK(c, hipMemcpyAsync(c->dcoef, hc, 1024 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_mupdate2(c, V, n, j, c->dcoef, c->dcoef + 512, 1.0 / rho, cvj, 1.0 / rho, w, vj));
    for (int i = 0; i <= j; ++i) H[i + (size_t)j * ld] = h[i];
    H[j + 1 + (size_t)j * ld] = 1.0;  // w holds v_{j+1} unnormalized (finished at the next step)
  }
  // second pass of the last vector: v_m <- (v_m - V s)/rho
  double* vm = V + (int64_t)m * n;
  HIPCHK(c, launch_mdot(c, V, n, m + 1, vm, c->dres));
  if ((rc = read_results(c, m + 1))) return rc;
  sv.assign(c->hres, c->hres + m);
  double col = c->hres[m];
  for (int i = 0; i < m; ++i) col += H[i + (size_t)(m - 1) * ld] * H[i + (size_t)(m - 1) * ld];
  double rho = 0.0;
  if (!finish_coeffs(m, sv.data(), c->hres[m], &rho)) {
    for (int cc = 0; cc < m; ++cc) H[m + (size_t)cc * ld] = 0.0;
    *kout = m;
    return KV_OK;
  }
  double* hc = c->hcoef;
  for (int i = 0; i < m; ++i) hc[i] = sv[i];
  HIPCHK(c, hipMemcpyAsync(c->dcoef, hc, m * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_mupdate(c, V, n, m, c->dcoef, vm));
  if ((rc = lincomb(c, 1, {1.0 / rho}, {vm}, vm))) return rc;
  *kout = m;
  (void)col;
  return KV_OK;
}

// ---- Ritz data -----------------------------------------------------------------------
struct Ritz {
  std::vector<std::complex<double>> vals;
  std::vector<int> sel;                                 // wanted, in output order
  std::vector<std::vector<std::complex<double>>> vecs;  // coefficient vectors of sel
  std::vector<double> res;                              // residual estimates of sel
};

std::vector<int> order_leading(const std::vector<std::complex<double>>& v) {
  std::vector<int> idx(v.size());
  for (size_t i = 0; i < v.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (v[a].real() != v[b].real()) return v[a].real() > v[b].real();
    return v[a].imag() > v[b].imag();
  });
  return idx;
}

std::vector<int> wanted_set(const std::vector<std::complex<double>>& v, int k) {
  std::vector<int> idx = order_leading(v);
  std::vector<int> sel(idx.begin(), idx.begin() + std::min<size_t>(k, idx.size()));
  if ((size_t)k < idx.size() && !sel.empty()) {
    const auto last = v[sel.back()];
    if (last.imag() > 0 && std::abs(v[idx[k]] - std::conj(last)) <= 1e-12 * std::max(1.0, std::abs(last)))
      sel.push_back(idx[k]);
  }
  return sel;
}

// Eigen-decomposition of H_k on the device; Ritz residuals h_{k+1,k} |e_k^T s|.
// The k values of smallest (or largest) modulus, extended by one when that
// would split a conjugate pair.
std::vector<int> modulus_set(const std::vector<std::complex<double>>& v, int k, bool largest) {
  std::vector<int> idx(v.size());
  for (size_t i = 0; i < v.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (std::abs(v[a]) != std::abs(v[b])) return largest ? std::abs(v[a]) > std::abs(v[b]) : std::abs(v[a]) < std::abs(v[b]);
    return v[a].imag() > v[b].imag();
  });
  std::vector<int> sel(idx.begin(), idx.begin() + std::min<size_t>(k, idx.size()));
  if (!sel.empty() && (size_t)k < idx.size()) {
    const auto last = v[sel.back()];
    if (last.imag() != 0.0) {
      bool partner = false;
      for (int i : sel) partner = partner || (i != sel.back() && std::abs(v[i] - std::conj(last)) <= 1e-12 * std::max(1.0, std::abs(last)));
      if (!partner)
        for (size_t q = k; q < idx.size(); ++q)
          if (std::abs(v[idx[q]] - std::conj(last)) <= 1e-12 * std::max(1.0, std::abs(last))) {
            sel.push_back(idx[q]);
            break;
          }
    }
  }
  return sel;
}

// Which Ritz values ritz() selects: largest real part first (the leading
// eigenvalues), smallest modulus (harmonic values of deflated GMRES) or
// largest modulus (the dominant values of a transformed operator).
enum { SEL_LEADING = 0, SEL_SMALLEST = 1, SEL_LARGEST = 2 };

int ritz(kv_ctx* c, const std::vector<double>& H, int m, int k, int n_eigs, Ritz& out, int order = SEL_LEADING) {
  // device layout: Hk (k*k) | Hcopy (k*k) | wr k | wi k | lr, li (k each) | vr, vi (k*k) | info | cwork
  const size_t kk = (size_t)k * k;
  int rc;
  double* d = c->hess;  // hess_area(k, n_eigs + 1) doubles, bound by the Arnoldi call
  double *dH = d, *dHc = d + kk, *dwr = d + 2 * kk, *dwi = dwr + k, *dlr = dwi + k, *dli = dlr + k;
  double *dvr = dli + k, *dvi = dvr + kk;
  int* dinfo = reinterpret_cast<int*>(dvi + kk);
  double* dcw = dvi + kk + 2;
  std::vector<double> Hk(kk);
  for (int r = 0; r < k; ++r)
    for (int cc = 0; cc < k; ++cc) Hk[(size_t)r * k + cc] = H[r + (size_t)cc * (m + 1)];
  if ((rc = upload(c, dH, Hk.data(), kk * sizeof(double)))) return rc;
  HIPCHK(c, hipMemcpyAsync(dHc, dH, kk * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, launch_hessenberg_values(c->stream, dHc, k, dwr, dwi, dinfo));
  std::vector<double> wr(k), wi(k);
  int info = 0;
  HIPCHK(c, hipMemcpyAsync(wr.data(), dwr, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(wi.data(), dwi, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info & 1) return fail(c, KV_ENOCONV, "Hessenberg QR did not converge");
  if (info & 2) ++c->relaxed_qr;  // a nearly defective cluster deflated at sqrt(eps)
  out.vals.resize(k);
  for (int i = 0; i < k; ++i) out.vals[i] = {wr[i], wi[i]};
  out.sel = order == SEL_LEADING ? wanted_set(out.vals, n_eigs) : modulus_set(out.vals, n_eigs, order == SEL_LARGEST);
  const int ns = (int)out.sel.size();
  std::vector<double> lr(ns), li(ns);
  for (int q = 0; q < ns; ++q) {
    lr[q] = out.vals[out.sel[q]].real();
    li[q] = out.vals[out.sel[q]].imag();
  }
  if ((rc = upload(c, dlr, lr.data(), ns * sizeof(double)))) return rc;
  if ((rc = upload(c, dli, li.data(), ns * sizeof(double)))) return rc;
  HIPCHK(c, launch_hessenberg_vectors(c->stream, dH, k, dlr, dli, ns, dcw, dvr, dvi));
  std::vector<double> vr((size_t)ns * k), vi((size_t)ns * k);
  HIPCHK(c, hipMemcpyAsync(vr.data(), dvr, vr.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(vi.data(), dvi, vi.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double hk = (k < m || H.size() > 0) ? H[k + (size_t)(k - 1) * (m + 1)] : 0.0;
  out.vecs.assign(ns, std::vector<std::complex<double>>(k));
  out.res.assign(ns, 0.0);
  for (int q = 0; q < ns; ++q) {
    // phase convention: unit 2-norm, largest-modulus component real positive
    int imax = 0;
    double amax = -1;
    for (int r = 0; r < k; ++r) {
      const double a = std::hypot(vr[(size_t)q * k + r], vi[(size_t)q * k + r]);
      if (a > amax + 1e-14 * amax) {
        amax = a;
        imax = r;
      }
    }
    const std::complex<double> ph =
        std::conj(std::complex<double>(vr[(size_t)q * k + imax], vi[(size_t)q * k + imax])) / amax;
    for (int r = 0; r < k; ++r) out.vecs[q][r] = std::complex<double>(vr[(size_t)q * k + r], vi[(size_t)q * k + r]) * ph;
    out.res[q] = std::fabs(hk) * std::abs(out.vecs[q][k - 1]);
  }
  return KV_OK;
}

// ---- Chebyshev helpers (ellipse and degree) ------------------------------------------------
// Ellipse (centre d, real semi-axis a, imaginary semi-axis b, c^2 = a^2 - b^2)
// symmetric about the real axis that encloses the unwanted Ritz values and
// stays left of the wanted ones: right end halfway between the largest
// unwanted and the smallest wanted real part, left end 1% of the unwanted
// real range beyond the smallest unwanted real part, b the smallest
// semi-axis that then encloses every unwanted value.
void ellipse(const std::vector<std::complex<double>>& unw, double wanted_min_re, double* d, double* a, double* b,
             double* c2) {
  double rmin = 1e300, rmax = -1e300;
  for (auto& z : unw) {
    rmin = std::min(rmin, z.real());
    rmax = std::max(rmax, z.real());
  }
  const double span = std::max(rmax - rmin, 1e-300);
  const double gap = wanted_min_re - rmax;
  const double right = gap > 0 ? rmax + 0.5 * gap : rmax + 1e-3 * span;
  const double left = rmin - 0.01 * span;
  *d = 0.5 * (left + right);
  *a = 0.5 * (right - left);
  double b2 = 0.0;
  for (auto& z : unw) {
    const double t = std::pow((z.real() - *d) / *a, 2);
    b2 = std::max(b2, z.imag() * z.imag() / (1.0 - t));
  }
  *b = std::sqrt(b2);
  *c2 = (*a) * (*a) - b2;
}

// Growth per degree of the ellipse's Chebyshev polynomial at z (from the
// centre) against its size on the ellipse: the larger root of w^2 - 2zw + c^2.
double growth_rate(std::complex<double> z, double a, double b, double c2) {
  const std::complex<double> s = std::sqrt(z * z - c2);
  return std::max(std::abs(z + s), std::abs(z - s)) / (a + b);
}

// Smallest degree with growth 1e6 at wr, at most dmax.
int cheb_degree(double wr, double a, double b, double c2, int dmax) {
  const double ratio = growth_rate(wr, a, b, c2);
  if (ratio <= 1.0 + 1e-12) return 0;
  const int d = (int)std::ceil(std::log(1e6) / std::log(ratio));
  return std::min(dmax, std::max(1, d));
}

}  // namespace

// Solves M t = b in place (b <- t) for a small dense complex M (row-major,
// nn x nn) by Gaussian elimination with partial pivoting; false if singular.
static bool solve_small(std::vector<std::complex<double>> M, std::vector<std::complex<double>>& b, int nn) {
  for (int col = 0; col < nn; ++col) {
    int piv = col;
    for (int r = col + 1; r < nn; ++r)
      if (std::abs(M[(size_t)r * nn + col]) > std::abs(M[(size_t)piv * nn + col])) piv = r;
    if (!(std::abs(M[(size_t)piv * nn + col]) > 0)) return false;
    if (piv != col) {
      for (int cc = 0; cc < nn; ++cc) std::swap(M[(size_t)piv * nn + cc], M[(size_t)col * nn + cc]);
      std::swap(b[piv], b[col]);
    }
    for (int r = col + 1; r < nn; ++r) {
      const std::complex<double> f = M[(size_t)r * nn + col] / M[(size_t)col * nn + col];
      for (int cc = col; cc < nn; ++cc) M[(size_t)r * nn + cc] -= f * M[(size_t)col * nn + cc];
      b[r] -= f * b[col];
    }
  }
  for (int r = nn - 1; r >= 0; --r) {
    for (int cc = r + 1; cc < nn; ++cc) b[r] -= M[(size_t)r * nn + cc] * b[cc];
    b[r] /= M[(size_t)r * nn + r];
  }
  return true;
}

// Eigenvectors of the output values into evecs (rows of n values; a pair as
// its real part, then its imaginary part).  A value found with nl vectors of
// L deflated has a Ritz vector y of the deflated operator; its eigenvector of
// A is x = y + L t with (theta - R) t = L^T W A y, R = L^T W A L over those nl
// vectors (A L = L R for the locked invariant subspaces).  Each x is scaled
// to unit W-norm; a complex x is turned by a phase so that its real and
// imaginary parts are W-orthogonal, the real part the longer.  zp, zc, tmp:
// scratch vectors.  Adds the matvecs used to *matvecs.
static int write_eigenvectors(kv_ctx* c, const double* L, const std::vector<int>& out,
                              const std::vector<std::complex<double>>& vals, const std::vector<const double*>& src_re,
                              const std::vector<const double*>& src_im, const std::vector<int>& nl, double* evecs,
                              double* zp, double* zc, double* tmp, int* matvecs) {
  const int64_t n = c->g.n;
  const int nL = c->nlock;
  int rc;
  c->nlock = 0;  // A itself below, not deflated
  std::vector<double> R((size_t)nL * nL, 0.0);
  bool need_R = false;
  for (int v : nl) need_R = need_R || v > 0;
  for (int j = 0; need_R && j < nL; ++j) {
    if ((rc = matvec(c, L + (int64_t)j * n, tmp))) return rc;
    ++*matvecs;
    HIPCHK(c, launch_mdot(c, L, n, nL, tmp));
    if ((rc = read_results(c, nL))) return rc;
    for (int i = 0; i < nL; ++i) R[(size_t)i * nL + j] = c->hres[i];
  }
  for (size_t q = 0; q < out.size(); ++q) {
    const std::complex<double> th = vals[out[q]];
    if (th.imag() < 0) continue;  // written with its +Im member
    const bool cplx = th.imag() > 0;
    HIPCHK(c, hipMemcpyAsync(zp, src_re[q], n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (cplx) HIPCHK(c, hipMemcpyAsync(zc, src_im[q], n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    const int k = nl[q];
    if (k > 0) {
      std::vector<std::complex<double>> rhs(k), M((size_t)k * k);
      for (int part = 0; part < (cplx ? 2 : 1); ++part) {
        if ((rc = matvec(c, part == 0 ? zp : zc, tmp))) return rc;
        ++*matvecs;
        HIPCHK(c, launch_mdot(c, L, n, k, tmp));
        if ((rc = read_results(c, k))) return rc;
        for (int i = 0; i < k; ++i) rhs[i] += part == 0 ? std::complex<double>(c->hres[i], 0.0)
                                                       : std::complex<double>(0.0, c->hres[i]);
      }
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) M[(size_t)i * k + j] = (i == j ? th : 0.0) - R[(size_t)i * nL + j];
      if (!solve_small(M, rhs, k)) return fail(c, KV_ENOCONV, "eigenvector lift: singular locked block");
      std::vector<double> cr(k), ci(k);
      for (int i = 0; i < k; ++i) {
        cr[i] = -rhs[i].real();
        ci[i] = -rhs[i].imag();
      }
      if ((rc = upload(c, c->dres, cr.data(), k * sizeof(double)))) return rc;
      HIPCHK(c, launch_mupdate(c, L, n, k, c->dres, zp));
      if (cplx) {
        if ((rc = upload(c, c->dres, ci.data(), k * sizeof(double)))) return rc;
        HIPCHK(c, launch_mupdate(c, L, n, k, c->dres, zc));
      }
    }
    const double a = dot1(c, zp, zp, &rc);
    if (rc) return rc;
    double* row = evecs + (int64_t)q * n;
    if (!cplx) {
      if (!(a > 0)) return fail(c, KV_ENONFINITE, "zero eigenvector");
      if ((rc = lincomb(c, 1, {1.0 / std::sqrt(a)}, {zp}, row))) return rc;
      continue;
    }
    const double b = dot1(c, zc, zc, &rc);
    if (rc) return rc;
    const double ab = dot1(c, zp, zc, &rc);
    if (rc) return rc;
    if (!(a + b > 0)) return fail(c, KV_ENONFINITE, "zero eigenvector");
    double phi = 0.5 * std::atan2(-2.0 * ab, a - b);
    double cs = std::cos(phi), sn = std::sin(phi);
    if (a * cs * cs - 2.0 * ab * sn * cs + b * sn * sn < a * sn * sn + 2.0 * ab * sn * cs + b * cs * cs) {
      phi += 1.5707963267948966;  // pi / 2
      cs = std::cos(phi);
      sn = std::sin(phi);
    }
    const double inv = 1.0 / std::sqrt(a + b);
    if ((rc = lincomb(c, 2, {cs * inv, -sn * inv}, {zp, zc}, row))) return rc;
    if ((rc = lincomb(c, 2, {sn * inv, cs * inv}, {zp, zc}, row + n))) return rc;
  }
  c->nlock = nL;
  return KV_OK;
}

// =============================================================================================
extern "C" {

int kv_create(const kv_params* p, void* hip_stream, kv_ctx** out) {
  if (!p || !out) return KV_EINVAL;
  *out = nullptr;
  if (p->nx < 2 || p->ny < 2 || p->nz < 2 || !p->xf || !p->yf || !p->zf || !(p->Gr >= 0) || !(p->Pr > 0))
    return KV_EINVAL;
  if (p->nx > 4096 || p->ny > 4096 || p->nz > 4096) return KV_EINVAL;
  kv_ctx* c = new (std::nothrow) kv_ctx();
  if (!c) return KV_ENOMEM;
  HostAxis ax[3];
  const double* faces[3] = {p->xf, p->yf, p->zf};
  const int ns[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    if (!build_axis(faces[a], ns[a], ax[a], c->err)) {
      delete c;
      return KV_EINVAL;
    }
    c->hf[a].assign(faces[a], faces[a] + ns[a] + 1);
  }
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return KV_EDEVICE;
  }
  Grid& g = c->g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  const int64_t nx = g.nx, ny = g.ny, nz = g.nz;
  g.ou = 0;
  g.ov = nz * ny * (nx - 1);
  g.ow = g.ov + nz * (ny - 1) * nx;
  g.oT = g.ow + (nz - 1) * ny * nx;
  g.n = g.oT + nz * ny * nx;
  c->ncell = nx * ny * nz;
  c->Gr = p->Gr;
  c->Pr = p->Pr;
  if (p->Gr > 0) {
    g.nu = 1.0 / std::sqrt(p->Gr);
    g.kappa = 1.0 / (p->Pr * std::sqrt(p->Gr));
    g.beta = 1.0;
  } else {
    g.nu = 1.0;
    g.kappa = 1.0 / p->Pr;
    g.beta = 0.0;
  }
  g.null3 = (int)(((int64_t)ax[2].null_idx * ny + ax[1].null_idx) * nx + ax[0].null_idx);
  // metrics: per axis 10 arrays of n+1 doubles
  size_t per_axis[3], total = 0;
  for (int a = 0; a < 3; ++a) {
    per_axis[a] = 10 * (size_t)(ns[a] + 1);
    total += per_axis[a];
  }
  std::vector<double> hm(total, 0.0);
  size_t o = 0;
  size_t offs[3][10];
  for (int a = 0; a < 3; ++a) {
    const std::vector<double>* arrs[10] = {&ax[a].h,  &ax[a].ih,  &ax[a].id, &ax[a].wlo, &ax[a].whi,
                                           &ax[a].sq, &ax[a].isq, &ax[a].dd, &ax[a].lam, &ax[a].c};
    for (int q = 0; q < 10; ++q) {
      offs[a][q] = o;
      std::copy(arrs[q]->begin(), arrs[q]->end(), hm.begin() + o);
      o += ns[a] + 1;
    }
  }
  auto cleanup = [&](int code, const char* msg) {
    kv_destroy(c);
    (void)msg;
    return code;
  };
  if (hipMalloc(&c->metric, total * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "metric");
  if (hipMemcpy(c->metric, hm.data(), total * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(KV_EDEVICE, "metric copy");
  for (int a = 0; a < 3; ++a) {
    Axis& A = g.ax[a];
    A.n = ns[a];
    const double* base = c->metric;
    A.h = base + offs[a][0];
    A.ih = base + offs[a][1];
    A.id = base + offs[a][2];
    A.wlo = base + offs[a][3];
    A.whi = base + offs[a][4];
    A.sq = base + offs[a][5];
    A.isq = base + offs[a][6];
    A.dd = base + offs[a][7];
    A.lam = base + offs[a][8];
    A.c = base + offs[a][9];
    const size_t nn = ax[a].Q.size();
    // the split kernels address a cell field with 32-bit byte offsets
    c->split[a] = (ax[a].split && c->ncell * 8 < ((int64_t)1 << 31)) ? 1 : 0;
    if (ax[a].split && !c->split[a]) {
      // rebuild this axis as a general (unsplit) basis
      HostAxis full;
      std::string e2;
      build_axis_general(faces[a], ns[a], full);
      ax[a] = full;
    }
    if (hipMalloc(&c->Qf[a], nn * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "Q");
    if (hipMalloc(&c->Qt[a], nn * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "Qt");
    if (hipMemcpy(c->Qf[a], ax[a].Q.data(), nn * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->Qt[a], ax[a].Qt.data(), nn * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(KV_EDEVICE, "Q copy");
    if (c->split[a]) {
      std::vector<float> q32(ax[a].Q.begin(), ax[a].Q.end()), qt32(ax[a].Qt.begin(), ax[a].Qt.end());
      if (hipMalloc(&c->Qf32[a], nn * sizeof(float)) != hipSuccess ||
          hipMalloc(&c->Qt32[a], nn * sizeof(float)) != hipSuccess)
        return cleanup(KV_ENOMEM, "Q32");
      if (hipMemcpy(c->Qf32[a], q32.data(), nn * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->Qt32[a], qt32.data(), nn * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(KV_EDEVICE, "Q32 copy");
    }
  }
  const int64_t rows = 2 * nz * ny + nz * (ny - 1) + (nz - 1) * ny;
  c->npart_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (rows + 3) / 4));
  // the Gram-Schmidt multi-dots carry 16-32 accumulators per thread and run
  // few waves per SIMD: up to four times as many blocks, but at least 8 rows
  // per wave, so that the per-block reduction of those accumulators stays
  // small beside the streaming on small grids (KV_MD_BLOCKS overrides, for
  // measurements)
  c->nmd_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (rows + 31) / 32));
  if (const char* mb = getenv("KV_MD_BLOCKS")) {
    const int v = atoi(mb);
    if (v >= 1 && v <= 8192) c->nmd_blocks = v;
  }
  if (hipMalloc(&c->X0, g.n * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "X0");
  if (hipMalloc(&c->cellA, c->ncell * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "cellA");
  if (hipMalloc(&c->cellB, c->ncell * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "cellB");
  if (hipMalloc(&c->part, (size_t)1024 * std::max(c->npart_blocks, c->nmd_blocks) * sizeof(double)) != hipSuccess)
    return cleanup(KV_ENOMEM, "part");
  if (hipMalloc(&c->dres, 1024 * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "dres");
  if (hipMalloc(&c->dcoef, 1024 * sizeof(double)) != hipSuccess) return cleanup(KV_ENOMEM, "dcoef");
  if (hipHostMalloc(&c->hcoef, 1024 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return cleanup(KV_ENOMEM, "hcoef");
  {
    // one pair of maxima per 64 x 4 block of the cell grid
    const int64_t cb = ((nx + 63) / 64) * ((ny + 3) / 4) * nz;
    c->cell_part_len = 2 * cb;
    if (hipMalloc(&c->cell_part, c->cell_part_len * sizeof(double)) != hipSuccess)
      return cleanup(KV_ENOMEM, "cell_part");
  }
  if (hipHostMalloc(&c->hres, 1024 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return cleanup(KV_ENOMEM, "hres");
  if (static_scratch_init(c->device) != 0) return cleanup(KV_EDEVICE, "static scratch");
  // kv_hessenberg_eigenvalues (m <= 400) and the interpolation tables of
  // kv_state_from_cells: small, fixed by the limits and the grid
  if (hipMalloc(&c->hess_small, (400 * 400 + 2 * 400 + 2) * sizeof(double)) != hipSuccess)
    return cleanup(KV_ENOMEM, "hess_small");
  {
    const int64_t nint = (2 * nx + 1) + (2 * ny + 1) + (2 * nz + 1);
    c->xfer_bytes = ((size_t)nint * sizeof(int) + 255) / 256 * 256 + (size_t)nint * sizeof(double);
    if (hipMalloc(&c->xfer, c->xfer_bytes) != hipSuccess) return cleanup(KV_ENOMEM, "xfer");
  }
  *out = c;
  return KV_OK;
}

int kv_destroy(kv_ctx* c) {
  if (!c) return KV_OK;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  hipFree(c->metric);
  for (int a = 0; a < 3; ++a) {
    hipFree(c->Qf[a]);
    hipFree(c->Qt[a]);
    hipFree(c->Qf32[a]);
    hipFree(c->Qt32[a]);
  }
  hipFree(c->cell_part);
  hipFree(c->X0);
  hipFree(c->cellA);
  hipFree(c->cellB);
  hipFree(c->part);
  hipFree(c->dres);
  hipFree(c->dcoef);
  if (c->hres) hipHostFree(c->hres);
  if (c->hcoef) hipHostFree(c->hcoef);
  for (auto& m : c->ev_marks) {
    hipEventDestroy(m.second.first);
    hipEventDestroy(m.second.second);
  }
  for (auto e : c->ev_pool) hipEventDestroy(e);
  hipFree(c->hess_small);
  hipFree(c->xfer);
  hipFree(c->pc_mem);
  delete c;
  return KV_OK;
}

int kv_layout(const kv_ctx* c, int64_t* n, int64_t off[5]) {
  if (!c) return KV_EINVAL;
  if (n) *n = c->g.n;
  if (off) {
    off[0] = c->g.ou;
    off[1] = c->g.ov;
    off[2] = c->g.ow;
    off[3] = c->g.oT;
    off[4] = c->g.n;
  }
  return KV_OK;
}

int kv_set_base_flow(kv_ctx* c, const double* X0) {
  if (!c) return KV_EINVAL;
  if (!X0) return fail(c, KV_EINVAL, "null base flow");
  int rc = check_finite(c, X0, c->g.n, "base flow");
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->X0, X0, c->g.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->has_base = true;
  return KV_OK;
}

int kv_apply_jacobian(kv_ctx* c, const double* x, double* y, unsigned flags) {
  if (!c) return KV_EINVAL;
  if (!x || !y || x == y) return fail(c, KV_EINVAL, "x and y must be distinct device vectors");
  if (flags & ~(unsigned)(KV_PROJECT | KV_MIXED)) return fail(c, KV_EINVAL, "unsupported flags");
  if (!c->has_base) return fail(c, KV_ESTATE, "no base flow");
  if ((flags & KV_PROJECT) && !((flags & KV_MIXED) && mixed_ok(c))) return apply_projected(c, x, y);
  int rc = apply_operator(c, x, y);
  if (rc) return rc;
  if (flags & KV_PROJECT) return project_mixed(c, y, nullptr, nullptr);
  return KV_OK;
}

int kv_project(kv_ctx* c, double* y, unsigned flags, double* div_max, int* sweeps) {
  if (!c) return KV_EINVAL;
  if (!y) return fail(c, KV_EINVAL, "null vector");
  if (flags & ~(unsigned)(KV_PROJECT | KV_MIXED)) return fail(c, KV_EINVAL, "unsupported flags");
  if ((flags & KV_MIXED) && mixed_ok(c)) return project_mixed(c, y, div_max, sweeps);
  int rc = project_inplace(c, y);
  if (rc) return rc;
  if (sweeps) *sweeps = 1;
  if (div_max) {
    HIPCHK(c, launch_div_measure(c, y));
    if ((rc = read_results(c, 2))) return rc;
    *div_max = c->hres[1] > 0 ? c->hres[0] / c->hres[1] : 0.0;
  }
  return KV_OK;
}

int kv_residual(kv_ctx* c, double* F, double* norm) {
  if (!c) return KV_EINVAL;
  if (!F) return fail(c, KV_EINVAL, "null output");
  if (!c->has_base) return fail(c, KV_ESTATE, "no base flow");
  HIPCHK(c, launch_operator(c, c->X0, c->X0, F, 1));
  int rc = project_inplace(c, F);
  if (rc) return rc;
  if (norm) {
    double v = dot1(c, F, F, &rc);
    if (rc) return rc;
    *norm = std::sqrt(std::max(0.0, v));
  }
  return KV_OK;
}

int kv_dot(kv_ctx* c, const double* a, const double* b, double* out) {
  if (!c) return KV_EINVAL;
  if (!a || !b || !out) return fail(c, KV_EINVAL, "null argument");
  int rc;
  *out = dot1(c, a, b, &rc);
  return rc;
}

int kv_axpby(kv_ctx* c, double a, const double* x, double b, double* y) {
  if (!c) return KV_EINVAL;
  if (!x || !y) return fail(c, KV_EINVAL, "null argument");
  if (!std::isfinite(a) || !std::isfinite(b)) return fail(c, KV_EINVAL, "non-finite coefficient");
  return lincomb(c, 2, {a, b}, {x, y}, y);
}

int kv_symmetry_project(kv_ctx* c, const double* x, double* y, unsigned sym) {
  if (!c) return KV_EINVAL;
  if (!x || !y) return fail(c, KV_EINVAL, "null argument");
  int er = 0, eo = 0, rc;
  if ((rc = check_sym(c, sym, &er, &eo))) return rc;
  HIPCHK(c, launch_symmetry_class(c, x, y, er, eo));
  return KV_OK;
}

int kv_symmetry_measures(kv_ctx* c, const double* X, double out[3]) {
  if (!c) return KV_EINVAL;
  if (!X || !out) return fail(c, KV_EINVAL, "null argument");
  HIPCHK(c, launch_symmetry(c, X));
  int rc = read_results(c, 3);
  if (rc) return rc;
  for (int q = 0; q < 3; ++q) out[q] = c->hres[q];
  return KV_OK;
}

// ---- Newton correction: BiCGstab(2), continued by GMRES(m) -------------------------------
static void hessenberg_keep_last(std::vector<double>& A, int m, std::vector<double>& Z);

// min || cv - Hb y || over y for a (k+1) x k matrix Hb (column-major, leading
// dimension ld) by Householder QR on the host; res = cv - Hb y.
static void lsq_solve(const std::vector<double>& Hb, int ld, int k, const std::vector<double>& cv,
                      std::vector<double>& y, std::vector<double>& res) {
  const int rows = k + 1;
  std::vector<double> R((size_t)rows * k), q(cv.begin(), cv.begin() + rows), v(rows);
  for (int cc = 0; cc < k; ++cc)
    for (int r = 0; r < rows; ++r) R[(size_t)r * k + cc] = Hb[r + (size_t)cc * ld];
  for (int cc = 0; cc < k; ++cc) {
    double nrm = 0.0;
    for (int r = cc; r < rows; ++r) nrm += R[(size_t)r * k + cc] * R[(size_t)r * k + cc];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double x0 = R[(size_t)cc * k + cc];
    const double alpha = x0 > 0 ? -nrm : nrm;
    double vv = 0.0;
    for (int r = cc; r < rows; ++r) {
      v[r] = R[(size_t)r * k + cc] - (r == cc ? alpha : 0.0);
      vv += v[r] * v[r];
    }
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    for (int c2 = cc; c2 < k; ++c2) {
      double t = 0.0;
      for (int r = cc; r < rows; ++r) t += v[r] * R[(size_t)r * k + c2];
      t *= beta;
      for (int r = cc; r < rows; ++r) R[(size_t)r * k + c2] -= t * v[r];
    }
    double t = 0.0;
    for (int r = cc; r < rows; ++r) t += v[r] * q[r];
    t *= beta;
    for (int r = cc; r < rows; ++r) q[r] -= t * v[r];
  }
  y.assign(k, 0.0);
  for (int r = k - 1; r >= 0; --r) {
    double acc = q[r];
    for (int c2 = r + 1; c2 < k; ++c2) acc -= R[(size_t)r * k + c2] * y[c2];
    const double d = R[(size_t)r * k + r];
    y[r] = d != 0.0 ? acc / d : 0.0;
  }
  res.assign(rows, 0.0);
  for (int r = 0; r < rows; ++r) {
    double acc = cv[r];
    for (int cc = 0; cc < k; ++cc) acc -= Hb[r + (size_t)cc * ld] * y[cc];
    res[r] = acc;
  }
}

// Solves M^T f = e (M k x k column-major ld, e = last unit vector) by
// Gaussian elimination with partial pivoting; false if singular.
static bool solve_transposed_last(const std::vector<double>& Hb, int ld, int k, std::vector<double>& f) {
  std::vector<double> A((size_t)k * k);
  for (int r = 0; r < k; ++r)
    for (int cc = 0; cc < k; ++cc) A[(size_t)r * k + cc] = Hb[cc + (size_t)r * ld];  // A = M^T
  f.assign(k, 0.0);
  f[k - 1] = 1.0;
  for (int col = 0; col < k; ++col) {
    int piv = col;
    for (int r = col + 1; r < k; ++r)
      if (std::fabs(A[(size_t)r * k + col]) > std::fabs(A[(size_t)piv * k + col])) piv = r;
    if (!(std::fabs(A[(size_t)piv * k + col]) > 0)) return false;
    if (piv != col) {
      for (int cc = 0; cc < k; ++cc) std::swap(A[(size_t)piv * k + cc], A[(size_t)col * k + cc]);
      std::swap(f[piv], f[col]);
    }
    for (int r = col + 1; r < k; ++r) {
      const double t = A[(size_t)r * k + col] / A[(size_t)col * k + col];
      if (t == 0.0) continue;
      for (int cc = col; cc < k; ++cc) A[(size_t)r * k + cc] -= t * A[(size_t)col * k + cc];
      f[r] -= t * f[col];
    }
  }
  for (int r = k - 1; r >= 0; --r) {
    for (int cc = r + 1; cc < k; ++cc) f[r] -= A[(size_t)r * k + cc] * f[cc];
    f[r] /= A[(size_t)r * k + r];
  }
  return true;
}

// Restarted GMRES(m) on A x = b from the current x (A = op_apply), with
// deflated restarting when c->gmres_defl > 0 (Morgan's GMRES-DR): after a
// full cycle the harmonic Ritz vectors of the gmres_defl values of smallest
// modulus (eigenvalues of H_m + h^2 H_m^-T e_m e_m^T) and the residual
// vector start the next cycle, so the few eigenvalues of the operator near
// zero -- the weakly damped modes of a steady branch near a Hopf point --
// stay in the space instead of being rebuilt every cycle.  The recursive
// residual estimate ends a cycle; the true residual b - A x confirms it.
// V: the basis (m + 1 vectors).  x_zero: x is 0 on entry, so the first
// residual is b itself (no operator application).
static int gmres_solve(kv_ctx* c, double* V, const double* b, double bnorm, double* x, double tol, int m, int budget,
                       int* used, int* cycles, double* relres, bool x_zero = false) {
  const int64_t n = c->g.n;
  int rc;
  std::vector<double> H, cv, y, res;
  // deflated restarts use the Hessenberg area, which a transformed Arnoldi
  // around an inner solve holds
  const int kd = c->st_inner ? 0 : std::min(c->gmres_defl, std::min(m - 2, 62));
  bool fresh = true;
  int j0 = 0;
  for (;;) {
    if (fresh) {
      // r = b - A x into V[0]
      if (x_zero) {
        HIPCHK(c, hipMemcpyAsync(V, b, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        x_zero = false;
      } else {
        if ((rc = op_apply(c, x, V))) return rc;
        ++*used;
        if ((rc = lincomb(c, 2, {1.0, -1.0}, {b, V}, V))) return rc;
      }
      double beta = std::sqrt(std::max(0.0, dot1(c, V, V, &rc)));
      if (rc) return rc;
      *relres = bnorm > 0 ? beta / bnorm : 0.0;
      if (!std::isfinite(beta)) return fail(c, KV_ENONFINITE, "non-finite GMRES residual");
      if (beta <= tol * bnorm) return KV_OK;
      if (*used + 2 > budget) return KV_ENOCONV;
      if ((rc = lincomb(c, 1, {1.0 / beta}, {V}, V))) return rc;
      cv.assign(1, beta);
      j0 = 0;
    }
    const int mm = std::max(j0 + 1, std::min(m, budget - *used - 1));
    int k = 0, mv = 0;
    if ((rc = arnoldi(c, V, mm, H, &k, &mv, j0))) return rc;
    *used += mv;
    const int ld = mm + 1;
    cv.resize(k + 1, 0.0);
    lsq_solve(H, ld, k, cv, y, res);
    // x += V y  (mupdate subtracts, so pass -y)
    std::vector<double> ny(k);
    for (int i = 0; i < k; ++i) ny[i] = -y[i];
    if ((rc = upload(c, c->dres, ny.data(), k * sizeof(double)))) return rc;
    HIPCHK(c, launch_mupdate(c, V, n, k, c->dres, x));
    ++*cycles;
    double rn = 0.0;
    for (double t : res) rn += t * t;
    rn = std::sqrt(rn);
    *relres = bnorm > 0 ? rn / bnorm : 0.0;
    if (rn <= tol * bnorm || kd == 0 || k < mm || mm < kd + 2 || *used + 2 > budget) {
      fresh = true;  // plain restart (or the final check) from the true residual
      continue;
    }
    // deflated restart: harmonic Ritz vectors of the kd values nearest zero
    std::vector<double> f;
    const double hl = H[k + (size_t)(k - 1) * ld];
    if (!solve_transposed_last(H, ld, k, f)) {
      fresh = true;
      continue;
    }
    std::vector<double> Mr((size_t)k * k), Z;
    for (int r = 0; r < k; ++r)
      for (int cc = 0; cc < k; ++cc) Mr[(size_t)r * k + cc] = H[r + (size_t)cc * ld];
    for (int r = 0; r < k; ++r) Mr[(size_t)r * k + (k - 1)] += hl * hl * f[r];
    hessenberg_keep_last(Mr, k, Z);
    std::vector<double> Hh((size_t)ld * mm, 0.0);
    for (int r = 0; r < k; ++r)
      for (int cc = std::max(0, r - 1); cc < k; ++cc) Hh[r + (size_t)cc * ld] = Mr[(size_t)r * k + cc];
    Ritz hz;
    if ((rc = ritz(c, Hh, mm, k, kd, hz, SEL_SMALLEST))) return rc;
    std::vector<std::vector<double>> Q;  // columns of length k + 1
    auto push = [&](std::vector<double> u) {
      for (int pass = 0; pass < 2; ++pass)
        for (const auto& qv : Q) {
          double d = 0.0;
          for (int r = 0; r <= k; ++r) d += qv[r] * u[r];
          for (int r = 0; r <= k; ++r) u[r] -= d * qv[r];
        }
      double nu = 0.0;
      for (double t : u) nu += t * t;
      nu = std::sqrt(nu);
      if (!(nu > 1e-12)) return false;
      for (double& t : u) t /= nu;
      Q.push_back(u);
      return true;
    };
    for (size_t q = 0; q < hz.sel.size() && (int)Q.size() < kd; ++q) {
      const auto th = hz.vals[hz.sel[q]];
      if (th.imag() < 0) continue;
      for (int part = 0; part < (th.imag() > 0 ? 2 : 1); ++part) {
        std::vector<double> u(k + 1, 0.0);
        for (int r = 0; r < k; ++r) {
          double acc = 0.0;
          for (int t = 0; t < k; ++t) acc += Z[(size_t)r * k + t] * (part == 0 ? hz.vecs[q][t].real() : hz.vecs[q][t].imag());
          u[r] = acc;
        }
        push(u);
      }
    }
    const int kq = (int)Q.size();
    if (kq < 1 || !push(res)) {  // the residual direction comes last
      fresh = true;
      continue;
    }
    // H_new = Q^T Hbar Q[0..k), cv_new = Q^T res, V <- V Q
    std::vector<double> HQ((size_t)(k + 1) * kq, 0.0);
    for (int cc = 0; cc < kq; ++cc)
      for (int r = 0; r <= k; ++r) {
        double acc = 0.0;
        for (int t = 0; t < k; ++t) acc += H[r + (size_t)t * ld] * Q[cc][t];
        HQ[(size_t)r * kq + cc] = acc;
      }
    std::vector<double> Hn((size_t)ld * mm, 0.0);
    for (int r = 0; r <= kq; ++r)
      for (int cc = 0; cc < kq; ++cc) {
        double acc = 0.0;
        for (int t = 0; t <= k; ++t) acc += Q[r][t] * HQ[(size_t)t * kq + cc];
        Hn[r + (size_t)cc * ld] = acc;
      }
    cv.assign(kq + 1, 0.0);
    for (int r = 0; r <= kq; ++r) {
      double acc = 0.0;
      for (int t = 0; t <= k; ++t) acc += Q[r][t] * res[t];
      cv[r] = acc;
    }
    std::vector<double> Wrow((size_t)(k + 1) * (kq + 1));
    for (int t = 0; t <= k; ++t)
      for (int cc = 0; cc <= kq; ++cc) Wrow[(size_t)t * (kq + 1) + cc] = Q[cc][t];
    if ((rc = upload(c, c->hess, Wrow.data(), Wrow.size() * sizeof(double)))) return rc;
    HIPCHK(c, launch_combine(c, V, n, k + 1, c->hess, kq + 1, V, n));
    H.swap(Hn);
    j0 = kq;
    fresh = false;
  }
}

namespace {
// Cayley transform C = (A - pole)^-1 (A - zero) of A = P J:
//   y = C x = x + (pole - zero) z,  (A - pole) z = x,
// z = M^-1 t from right-preconditioned restarted GMRES on (A - pole) M^-1 t
// = x from t = 0 (without a preconditioner z = t), to st_tol relative.  x
// and z stay in range(P) and in the symmetry class kept.
int cayley_apply(kv_ctx* c, const double* x, double* y) {
  const int64_t n = c->g.n;
  int rc = KV_OK;
  const double bn = std::sqrt(std::max(0.0, dot1(c, x, x, &rc)));
  if (rc) return rc;
  HIPCHK(c, launch_fill(c, n, 0.0, c->st_t));
  c->st_inner = true;
  c->pc_active = c->pc_kind != KV_PC_NONE;
  int used = 0, cyc = 0;
  double rr = 0.0;
  rc = gmres_solve(c, c->st_V, x, bn, c->st_t, c->st_tol, c->gmres_m, c->st_max_matvec, &used, &cyc, &rr, true);
  c->st_matvecs += used;
  ++c->st_solves;
  static const bool trace = [] {
    const char* ev = getenv("KV_ARNOLDI_TRACE");
    return ev && atoi(ev) != 0;
  }();
  if (trace) fprintf(stderr, "[cayley] inner solve %d: %d matvecs, relative residual %.3e\n", c->st_solves, used, rr);
  double* z = c->st_t;
  if (rc == KV_OK && c->pc_active) {
    rc = precond_apply(c, c->st_t, c->pc_tmp);
    z = c->pc_tmp;
  }
  c->st_inner = false;
  c->pc_active = false;
  if (rc == KV_ENOCONV) {
    char msg[160];
    snprintf(msg, sizeof msg, "spectral transform: inner solve at relative residual %.3e after %d matvecs", rr, used);
    return fail(c, KV_ENOCONV, msg);
  }
  if (rc) return rc;
  if (c->sym_ref || c->sym_rot) HIPCHK(c, launch_symmetry_class(c, z, z, c->sym_ref, c->sym_rot));
  return lincomb(c, 2, {1.0, c->st_pole - c->st_zero}, {x, z}, y);
}
}  // namespace

static int newton_correction(kv_ctx* c, const double* F, double tol, int max_matvec, const double* delta0,
                             double* delta, kv_solve_info* info);

int kv_newton_correction(kv_ctx* c, const double* F, double tol, int max_matvec, unsigned flags,
                         const double* delta0, double* delta, kv_solve_info* info) {
  if (!c) return KV_EINVAL;
  if (!F || !delta || F == delta) return fail(c, KV_EINVAL, "F and delta must be distinct device vectors");
  int er = 0, eo = 0, rc;
  if ((rc = check_sym(c, flags, &er, &eo))) return rc;
  if (!(tol > 0) || max_matvec < 4) return fail(c, KV_EINVAL, "bad tolerance or budget");
  if (!c->has_base) return fail(c, KV_ESTATE, "no base flow");
  if (delta0 == delta) return fail(c, KV_EINVAL, "delta0 must not alias delta");
  EigScope scope(c, er, eo, nullptr);  // matvec keeps the Krylov space in the class
  MixedScope mixed(c);
  c->pc_active = c->pc_kind != KV_PC_NONE;
  rc = newton_correction(c, F, tol, max_matvec, delta0, delta, info);
  c->pc_active = false;
  return rc;
}

// With the preconditioner the Krylov iterate x lives in the preconditioned
// space: delta = delta0 + M^-1 x.  Without it, delta = x.  Either way the
// result is projected once more (the Krylov combination is divergence-free
// only up to cancellation among its projected terms).
static int finish_delta(kv_ctx* c, double* x, bool has_d0) {
  if (c->pc_active) {
    int rc = precond_apply(c, x, c->pc_tmp);
    if (rc) return rc;
    if (has_d0) rc = lincomb(c, 2, {1.0, 1.0}, {c->pc_tmp, c->pc_d0}, x);
    else rc = lincomb(c, 1, {1.0}, {c->pc_tmp}, x);
    if (rc) return rc;
  }
  int rc = project_inplace(c, x);
  if (rc) return rc;
  if (c->sym_ref || c->sym_rot) HIPCHK(c, launch_symmetry_class(c, x, x, c->sym_ref, c->sym_rot));
  return KV_OK;
}

static int newton_correction(kv_ctx* c, const double* F, double tol, int max_matvec, const double* delta0,
                             double* delta, kv_solve_info* info) {
  const int64_t n = c->g.n;
  int rc;
  if ((rc = check_finite(c, F, n, "F"))) return rc;
  // BiCGstab(2) vectors and the GMRES(m) basis (and the preconditioner's
  // vectors) from the caller's workspace
  if ((rc = ws_bind(c, KV_WS_NEWTON, 0, 0))) return rc;
  double* W = c->ws;
  double *b = W, *rt = W + n, *r0 = W + 2 * n, *r1 = W + 3 * n, *r2 = W + 4 * n;
  double *u0 = W + 5 * n, *u1 = W + 6 * n, *u2 = W + 7 * n;
  double* r[3] = {r0, r1, r2};
  double* u[3] = {u0, u1, u2};
  double* x = delta;
  kv_solve_info inf{0, 0, 0, 0.0, 0};
  // b = -P F (in the symmetry class when one is kept)
  if ((rc = lincomb(c, 1, {-1.0}, {F}, b))) return rc;
  if ((rc = project_inplace(c, b))) return rc;
  if (c->sym_ref || c->sym_rot) HIPCHK(c, launch_symmetry_class(c, b, b, c->sym_ref, c->sym_rot));
  const double bnorm = std::sqrt(std::max(0.0, dot1(c, b, b, &rc)));
  if (rc) return rc;
  if (delta0 && c->pc_active) {
    // delta = delta0 + M^-1 x, x from 0: the residual of delta0 starts the solve
    HIPCHK(c, hipMemcpyAsync(c->pc_d0, delta0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if ((rc = matvec(c, c->pc_d0, r0))) return rc;
    ++inf.matvecs;
    if ((rc = lincomb(c, 2, {1.0, -1.0}, {b, r0}, r0))) return rc;
    HIPCHK(c, launch_fill(c, n, 0.0, x));
  } else if (delta0) {
    HIPCHK(c, hipMemcpyAsync(x, delta0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if ((rc = matvec(c, x, r0))) return rc;
    ++inf.matvecs;
    if ((rc = lincomb(c, 2, {1.0, -1.0}, {b, r0}, r0))) return rc;
  } else {
    HIPCHK(c, launch_fill(c, n, 0.0, x));
    HIPCHK(c, hipMemcpyAsync(r0, b, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
  if (bnorm == 0.0) {
    if (info) *info = inf;
    return finish_delta(c, x, delta0 != nullptr);
  }
  HIPCHK(c, hipMemcpyAsync(rt, r0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, launch_fill(c, n, 0.0, u0));
  double rho0 = 1.0, alpha = 0.0, omega = 1.0;
  double res = std::sqrt(std::max(0.0, dot1(c, r0, r0, &rc)));
  if (rc) return rc;
  double best = res;
  int best_cycle = 0;
  const double scale = bnorm * bnorm;
  enum { CONV, BREAK, STAG, MAXIT } status = CONV;
  for (;;) {
    if (res <= tol * bnorm) {
      status = CONV;
      break;
    }
    if (inf.cycles - best_cycle >= c->stall_cycles) {
      status = STAG;
      break;
    }
    if (inf.matvecs + 4 > max_matvec) {
      status = MAXIT;
      break;
    }
    rho0 = -omega * rho0;
    bool broke = false;
    for (int j = 0; j < 2 && !broke; ++j) {
      const double rho1 = dot1(c, r[j], rt, &rc);
      if (rc) return rc;
      if (std::fabs(rho0) <= 1e-300 * scale || rho1 == 0.0) {
        broke = true;
        break;
      }
      const double beta = alpha * rho1 / rho0;
      rho0 = rho1;
      for (int i = 0; i <= j; ++i)
        if ((rc = lincomb(c, 2, {1.0, -beta}, {r[i], u[i]}, u[i]))) return rc;
      if ((rc = op_apply(c, u[j], u[j + 1]))) return rc;
      ++inf.matvecs;
      const double gamma = dot1(c, u[j + 1], rt, &rc);
      if (rc) return rc;
      if (std::fabs(gamma) <= 1e-300 * scale) {
        broke = true;
        break;
      }
      alpha = rho0 / gamma;
      for (int i = 0; i <= j; ++i)
        if ((rc = lincomb(c, 2, {1.0, -alpha}, {r[i], u[i + 1]}, r[i]))) return rc;
      if ((rc = op_apply(c, r[j], r[j + 1]))) return rc;
      ++inf.matvecs;
      if ((rc = lincomb(c, 2, {1.0, alpha}, {x, u[0]}, x))) return rc;
    }
    if (broke) {
      status = BREAK;
      break;
    }
    // minimal-residual part over span{r1, r2}
    double d3[3];
    {
      const double* a[3] = {r1, r0, r2};
      const double* bb[3] = {r1, r1, r1};
      if ((rc = dots(c, 3, a, bb, d3))) return rc;
    }
    const double sigma1 = d3[0], g1p = d3[1] / sigma1, tau12 = d3[2] / sigma1;
    if ((rc = lincomb(c, 2, {1.0, -tau12}, {r2, r1}, r2))) return rc;
    double d2[2];
    {
      const double* a[2] = {r2, r0};
      const double* bb[2] = {r2, r2};
      if ((rc = dots(c, 2, a, bb, d2))) return rc;
    }
    const double sigma2 = d2[0], g2p = d2[1] / sigma2;
    const double g2 = g2p, g1 = g1p - tau12 * g2, g1pp = g2;
    omega = g2;
    if ((rc = lincomb(c, 3, {1.0, g1, g1pp}, {x, r0, r1}, x))) return rc;
    if ((rc = lincomb(c, 3, {1.0, -g2p, -g1p}, {r0, r2, r1}, r0))) return rc;
    if ((rc = lincomb(c, 3, {1.0, -g2, -g1}, {u0, u2, u1}, u0))) return rc;
    ++inf.cycles;
    res = std::sqrt(std::max(0.0, dot1(c, r0, r0, &rc)));
    if (rc) return rc;
    if (!std::isfinite(res)) {
      status = BREAK;
      break;
    }
    if (res < 0.9 * best) {
      best = res;
      best_cycle = inf.cycles;
    }
  }
  inf.relres = res / bnorm;
  if (status == BREAK || status == STAG) {
    inf.used_gmres = 1;
    int used = inf.matvecs, cyc = inf.cycles;
    double rr = inf.relres;
    // With the preconditioner and an initial iterate the Krylov unknown x
    // solves P J M^-1 x = b - P J delta0, whose right-hand side is the
    // initial residual: the shadow vector rt still holds it.
    const double* rhs = (c->pc_active && delta0) ? rt : b;
    // the basis follows the 8 BiCGstab(2) vectors (ws_bind, KV_WS_NEWTON)
    rc = gmres_solve(c, c->ws + 8 * n, rhs, bnorm, x, tol, c->gmres_m, max_matvec, &used, &cyc, &rr);
    inf.matvecs = used;
    inf.cycles = cyc;
    inf.relres = rr;
    if (c->pc_active) inf.precond = inf.matvecs - (delta0 ? 1 : 0);
    if (info) *info = inf;
    if (rc != KV_OK && rc != KV_ENOCONV) return rc;
    const int rf = finish_delta(c, x, delta0 != nullptr);
    if (rf) return rf;
    if (rc == KV_ENOCONV) return fail(c, KV_ENOCONV, "Newton correction: matvec budget exhausted");
    return KV_OK;
  }
  if (c->pc_active) inf.precond = inf.matvecs - (delta0 ? 1 : 0);
  if (info) *info = inf;
  const int rf = finish_delta(c, x, delta0 != nullptr);
  if (rf) return rf;
  if (status == MAXIT) return fail(c, KV_ENOCONV, "Newton correction: matvec budget exhausted");
  return KV_OK;
}

// ---- Stokes/heat preconditioner ------------------------------------------------------------
// 1-D operator -(H^-1 K) of kind HB_* along an axis with faces f (n cells):
// returns K (m x m, row-major) and the widths H (m values).
static void helm_operator(const std::vector<double>& f, int kind, std::vector<double>& K, std::vector<double>& H) {
  const int n = (int)f.size() - 1;
  std::vector<double> h(n), d(n + 1);
  for (int i = 0; i < n; ++i) h[i] = f[i + 1] - f[i];
  d[0] = 0.5 * h[0];
  d[n] = 0.5 * h[n - 1];
  for (int i = 1; i < n; ++i) d[i] = 0.5 * (h[i - 1] + h[i]);
  if (kind == HB_FD) {
    const int m = n - 1;  // interior face i + 1 sits between cells i and i + 1
    K.assign((size_t)m * m, 0.0);
    H.resize(m);
    for (int i = 0; i < m; ++i) {
      H[i] = d[i + 1];
      K[(size_t)i * m + i] = 1.0 / h[i] + 1.0 / h[i + 1];
      if (i + 1 < m) K[(size_t)i * m + i + 1] = K[(size_t)(i + 1) * m + i] = -1.0 / h[i + 1];
    }
    return;
  }
  K.assign((size_t)n * n, 0.0);
  H = h;
  for (int i = 0; i + 1 < n; ++i) {  // flux between centres i and i + 1 over the gap d[i + 1]
    const double t = 1.0 / d[i + 1];
    K[(size_t)i * n + i] += t;
    K[(size_t)(i + 1) * n + i + 1] += t;
    K[(size_t)i * n + i + 1] = K[(size_t)(i + 1) * n + i] = -t;
  }
  if (kind == HB_CD) {  // zero wall values at half-cell distance
    K[0] += 1.0 / d[0];
    K[(size_t)n * n - 1] += 1.0 / d[n];
  }
}

static int build_preconditioner(kv_ctx* c) {
  if (c->pc_mem) return KV_OK;
  size_t total = 0;
  int sizes[3][3];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      const int n = (int)c->hf[a].size() - 1;
      sizes[a][k] = k == HB_FD ? n - 1 : n;
      total += 4 * (size_t)sizes[a][k] * sizes[a][k] + sizes[a][k];
    }
  std::vector<double> host(total);
  size_t o = 0;
  size_t offs[3][3][5];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      const int m = sizes[a][k];
      std::vector<double> K, H, Q, lam;
      helm_operator(c->hf[a], k, K, H);
      std::vector<double> s(m), is(m);
      for (int i = 0; i < m; ++i) {
        s[i] = std::sqrt(H[i]);
        is[i] = 1.0 / s[i];
      }
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) K[(size_t)i * m + j] *= is[i] * is[j];
      jacobi_eigen(m, K, Q, lam);
      for (double& l : lam) l = std::max(l, 0.0);
      double* fwdB = host.data() + o;
      double* fwdA = fwdB + (size_t)m * m;
      double* invB = fwdA + (size_t)m * m;
      double* invA = invB + (size_t)m * m;
      double* lm = invA + (size_t)m * m;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          const double q = Q[(size_t)i * m + j];  // row i = position, column j = mode
          fwdB[(size_t)i * m + j] = s[i] * q;
          fwdA[(size_t)j * m + i] = s[i] * q;
          invB[(size_t)j * m + i] = is[i] * q;
          invA[(size_t)i * m + j] = is[i] * q;
        }
      for (int j = 0; j < m; ++j) lm[j] = lam[j];
      for (int q = 0; q < 5; ++q) offs[a][k][q] = o + (size_t)q * m * m;
      o += 4 * (size_t)m * m + m;
    }
  if (hipMalloc(&c->pc_mem, total * sizeof(double)) != hipSuccess) {
    c->pc_mem = nullptr;
    return fail(c, KV_ENOMEM, "preconditioner bases");
  }
  int rc = upload(c, c->pc_mem, host.data(), total * sizeof(double));
  if (rc) return rc;
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      HelmBasis& hb = c->hb[a][k];
      hb.n = sizes[a][k];
      hb.fwdB = c->pc_mem + offs[a][k][0];
      hb.fwdA = c->pc_mem + offs[a][k][1];
      hb.invB = c->pc_mem + offs[a][k][2];
      hb.invA = c->pc_mem + offs[a][k][3];
      hb.lam = c->pc_mem + offs[a][k][4];
    }
  return KV_OK;
}

// ---- time integration ------------------------------------------------------------------------
// Semi-implicit steps of Eqs. 1-6 with the library's operators: diffusion
// implicit through the Helmholtz solves of the Stokes/heat preconditioner,
// advection and buoyancy explicit, every step projected.  With F = P N(X)
// (diffusion included) and M_s^-1 = the preconditioner at shift s:
//   order 1:  X+ = X + M_{1/dt}^-1 F(X)
//   order 2 (SBDF2), s = 3/(2 dt):
//     X+ = 2X - X- + M_s^-1 [ (2s/3)(X- - X) + 2F(X) - F(X-) ]
// which is (3X+ - 4X + X-)/(2 dt) = 2E(X) - E(X-) + L X+ rewritten with
// E = N - L (L the homogeneous diffusion inside M; the inhomogeneous wall
// terms cancel).  Fixed points are exactly the steady states (M_s^-1 is
// W-positive definite on range(P)).
int kv_time_steps(kv_ctx* c, double dt, int nsteps, int start, double* X, double* Xprev) {
  if (!c) return KV_EINVAL;
  if (!X || !Xprev || X == Xprev) return fail(c, KV_EINVAL, "X and Xprev must be distinct device vectors");
  if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0 || (start != 0 && start != 1))
    return fail(c, KV_EINVAL, "bad time-step arguments");
  int rc;
  if ((rc = ws_bind(c, KV_WS_TIME_STEPS, 0, 0))) return rc;
  if ((rc = build_preconditioner(c))) return rc;
  const int64_t n = c->g.n;
  double* F = c->ws;
  double* Fp = c->ws + n;
  double* R = c->ws + 2 * n;
  const int kind0 = c->pc_kind;
  const double sig0 = c->pc_sigma;
  c->pc_kind = KV_PC_STOKES;
  auto restore = [&](int code) {
    c->pc_kind = kind0;
    c->pc_sigma = sig0;
    return code;
  };
  auto residual_into = [&](const double* Xs, double* out) -> int {
    HIPCHK(c, launch_operator(c, Xs, Xs, out, 1));
    return project_inplace(c, out);
  };
  if (nsteps > 0 && !start)
    if ((rc = residual_into(Xprev, Fp))) return restore(rc);
  for (int s = 0; s < nsteps; ++s) {
    if ((rc = residual_into(X, F))) return restore(rc);
    if (s == 0 && start) {
      c->pc_sigma = 1.0 / dt;
      if ((rc = precond_apply(c, F, R))) return restore(rc);
      HIPCHK(c, hipMemcpyAsync(Xprev, X, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      if ((rc = lincomb(c, 2, {1.0, 1.0}, {X, R}, X))) return restore(rc);
    } else {
      const double sg = 1.5 / dt;
      c->pc_sigma = sg;
      const double a = 2.0 * sg / 3.0;
      if ((rc = lincomb(c, 4, {a, -a, 2.0, -1.0}, {Xprev, X, F, Fp}, R))) return restore(rc);
      if ((rc = precond_apply(c, R, R))) return restore(rc);
      if ((rc = lincomb(c, 3, {2.0, -1.0, 1.0}, {X, Xprev, R}, R))) return restore(rc);
      HIPCHK(c, hipMemcpyAsync(Xprev, X, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(X, R, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    std::swap(F, Fp);  // F(X) of this step is F(X-) of the next
  }
  if (nsteps > 0 && (rc = check_finite(c, X, n, "time step"))) return restore(rc);
  return restore(KV_OK);
}

int kv_set_gmres_restart(kv_ctx* c, int m) {
  if (!c) return KV_EINVAL;
  if (m < 10 || m > 400) return fail(c, KV_EINVAL, "GMRES restart length must be in 10..400");
  c->gmres_m = m;
  return KV_OK;
}

int kv_workspace_size(const kv_ctx* c, int op, int krylov_dim, int n_eigs, size_t* bytes) {
  if (!c || !bytes) return KV_EINVAL;
  if (op < KV_WS_PROJECT_MIXED || op > KV_WS_TIME_STEPS) return KV_EINVAL;
  if (op == KV_WS_ARNOLDI && (krylov_dim < 2 || krylov_dim > 400 || n_eigs < 1 || n_eigs >= krylov_dim))
    return KV_EINVAL;
  *bytes = ws_need(c, op, krylov_dim, n_eigs);
  return KV_OK;
}

int kv_set_workspace(kv_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return KV_EINVAL;
  if ((dev_ptr == nullptr) != (bytes == 0)) return fail(c, KV_EINVAL, "workspace pointer and size must both be set or both be 0");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 8) return fail(c, KV_EINVAL, "workspace must be 8-byte aligned");
  c->ws = static_cast<double*>(dev_ptr);
  c->ws_bytes = bytes;
  c->ymix = c->pc_tmp = c->pc_d0 = c->pc_scr = c->hess = nullptr;
  return KV_OK;
}

int kv_set_gmres_deflation(kv_ctx* c, int k) {
  if (!c) return KV_EINVAL;
  if (k < 0 || k > 62) return fail(c, KV_EINVAL, "GMRES deflation must be in 0..62");
  c->gmres_defl = k;
  return KV_OK;
}

int kv_set_solver_projection(kv_ctx* c, unsigned flags) {
  if (!c) return KV_EINVAL;
  if (flags & ~(unsigned)KV_MIXED) return fail(c, KV_EINVAL, "unsupported flags");
  if ((flags & KV_MIXED) && !mixed_grid(c))
    return fail(c, KV_EINVAL, "the mixed projection needs mirror-symmetric axes of even size");
  c->solve_mixed_set = (flags & KV_MIXED) != 0;
  return KV_OK;
}

int kv_set_spectral_transform(kv_ctx* c, int kind, double pole, double zero, double inner_tol, int inner_max_matvec) {
  if (!c) return KV_EINVAL;
  if (kind == KV_ST_NONE) {
    c->st_kind = KV_ST_NONE;
    return KV_OK;
  }
  if (kind != KV_ST_CAYLEY) return fail(c, KV_EINVAL, "unknown spectral transform");
  if (!std::isfinite(pole) || !std::isfinite(zero) || pole == zero)
    return fail(c, KV_EINVAL, "the pole and zero of the Cayley transform must be finite and distinct");
  if (!(inner_tol > 0.0 && inner_tol < 1.0) || inner_max_matvec < 4)
    return fail(c, KV_EINVAL, "bad inner tolerance or budget");
  c->st_kind = kind;
  c->st_pole = pole;
  c->st_zero = zero;
  c->st_tol = inner_tol;
  c->st_max_matvec = inner_max_matvec;
  return KV_OK;
}

int kv_set_bicgstab_stall(kv_ctx* c, int cycles) {
  if (!c) return KV_EINVAL;
  if (cycles < 0 || cycles > 100000) return fail(c, KV_EINVAL, "stall cycles must be in 0..100000");
  c->stall_cycles = cycles;
  return KV_OK;
}

int kv_set_preconditioner(kv_ctx* c, int kind, double sigma) {
  if (!c) return KV_EINVAL;
  if (kind != KV_PC_NONE && kind != KV_PC_STOKES) return fail(c, KV_EINVAL, "unknown preconditioner");
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(c, KV_EINVAL, "sigma must be finite and >= 0");
  if (kind == KV_PC_STOKES) {
    const int rc = build_preconditioner(c);
    if (rc) return rc;
  }
  c->pc_kind = kind;
  c->pc_sigma = sigma;
  return KV_OK;
}

int kv_apply_preconditioner(kv_ctx* c, const double* x, double* y) {
  if (!c) return KV_EINVAL;
  if (!x || !y) return fail(c, KV_EINVAL, "null argument");
  if (c->pc_kind == KV_PC_NONE) return fail(c, KV_ESTATE, "no preconditioner set");
  int rc = ws_bind(c, KV_WS_APPLY_PRECONDITIONER, 0, 0);
  if (rc) return rc;
  return precond_apply(c, x, y);
}

// ---- transfers to and from the network grid --------------------------------------------
static bool affine_ok(const double shift[4], const double scale[4]) {
  if (!shift || !scale) return false;
  for (int q = 0; q < 4; ++q)
    if (!std::isfinite(shift[q]) || !std::isfinite(scale[q]) || scale[q] == 0.0) return false;
  return true;
}

int kv_cells_from_state(kv_ctx* c, const double* X, int factor, const double shift[4], const double scale[4],
                        float* out) {
  if (!c) return KV_EINVAL;
  if (!X || !out) return fail(c, KV_EINVAL, "null argument");
  if (factor < 1 || c->g.nx % factor || c->g.ny % factor || c->g.nz % factor)
    return fail(c, KV_EINVAL, "the grid sizes must be multiples of factor");
  if (!affine_ok(shift, scale)) return fail(c, KV_EINVAL, "shift/scale must be finite, scale nonzero");
  int rc;
  if ((rc = check_finite(c, X, c->g.n, "X"))) return rc;
  HIPCHK(c, launch_cells_from_state(c, X, factor, shift, scale, out));
  return KV_OK;
}

// For positions s (ascending) on [0, 1]: q = lower node in e (size r + 2)
// with q <= r, t = weight of node q + 1.
static void interp_table(const std::vector<double>& e, const double* s, int ns, int* q, double* t) {
  const int r = (int)e.size() - 2;
  for (int i = 0; i < ns; ++i) {
    int k = (int)(std::upper_bound(e.begin(), e.end(), s[i]) - e.begin()) - 1;
    k = std::max(0, std::min(k, r));
    q[i] = k;
    const double w = (s[i] - e[k]) / (e[k + 1] - e[k]);
    t[i] = std::max(0.0, std::min(1.0, w));
  }
}

static int state_from_cells(kv_ctx* c, const float* cells, const float* cells_ref, int rx, int ry, int rz,
                            const double* xc, const double* yc, const double* zc, const double shift[4],
                            const double scale[4], double* X) {
  if (!c) return KV_EINVAL;
  if (!cells || !X || !xc || !yc || !zc) return fail(c, KV_EINVAL, "null argument");
  if (rx < 1 || ry < 1 || rz < 1 || rx > 4096 || ry > 4096 || rz > 4096)
    return fail(c, KV_EINVAL, "network grid sizes must be in [1, 4096]");
  if (!affine_ok(shift, scale)) return fail(c, KV_EINVAL, "shift/scale must be finite, scale nonzero");
  const int r[3] = {rx, ry, rz};
  const double* cen[3] = {xc, yc, zc};
  std::vector<double> e[3];
  for (int a = 0; a < 3; ++a) {
    e[a].push_back(0.0);
    for (int i = 0; i < r[a]; ++i) e[a].push_back(cen[a][i]);
    e[a].push_back(1.0);
    for (size_t i = 1; i < e[a].size(); ++i)
      if (!(e[a][i] > e[a][i - 1])) return fail(c, KV_EINVAL, "network centres must increase strictly inside (0, 1)");
  }
  // tables: per axis faces (n+1) then centres (n); ints first, then doubles
  const int n3[3] = {c->g.nx, c->g.ny, c->g.nz};
  int64_t nint = 0;
  for (int a = 0; a < 3; ++a) nint += 2 * n3[a] + 1;
  const size_t dbl_off = ((size_t)nint * sizeof(int) + 255) / 256 * 256;
  const size_t bytes = dbl_off + (size_t)nint * sizeof(double);
  if (c->xfer_bytes < bytes) return fail(c, KV_EINVAL, "interpolation tables exceed their create-time size");
  std::vector<int> hq(nint);
  std::vector<double> ht(nint);
  const int* qp[6];
  const double* tp[6];
  int64_t o = 0;
  for (int a = 0; a < 3; ++a) {
    const int n = n3[a];
    std::vector<double> centres(n);
    for (int i = 0; i < n; ++i) centres[i] = 0.5 * (c->hf[a][i] + c->hf[a][i + 1]);
    interp_table(e[a], c->hf[a].data(), n + 1, hq.data() + o, ht.data() + o);
    qp[2 * a] = (const int*)c->xfer + o;
    tp[2 * a] = (const double*)((char*)c->xfer + dbl_off) + o;
    o += n + 1;
    interp_table(e[a], centres.data(), n, hq.data() + o, ht.data() + o);
    qp[2 * a + 1] = (const int*)c->xfer + o;
    tp[2 * a + 1] = (const double*)((char*)c->xfer + dbl_off) + o;
    o += n;
  }
  int rc;
  if ((rc = upload(c, c->xfer, hq.data(), nint * sizeof(int)))) return rc;
  if ((rc = upload(c, (char*)c->xfer + dbl_off, ht.data(), nint * sizeof(double)))) return rc;
  HIPCHK(c, launch_state_from_cells(c, cells, cells_ref, r, qp, tp, shift, scale, X));
  return KV_OK;
}

int kv_state_from_cells(kv_ctx* c, const float* cells, int rx, int ry, int rz, const double* xc, const double* yc,
                        const double* zc, const double shift[4], const double scale[4], double* X) {
  return state_from_cells(c, cells, nullptr, rx, ry, rz, xc, yc, zc, shift, scale, X);
}

int kv_state_add_cell_increment(kv_ctx* c, const float* cells, const float* cells_ref, int rx, int ry, int rz,
                                const double* xc, const double* yc, const double* zc, const double scale[4],
                                double* X) {
  if (!c) return KV_EINVAL;
  if (!cells_ref) return fail(c, KV_EINVAL, "null argument");
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  return state_from_cells(c, cells, cells_ref, rx, ry, rz, xc, yc, zc, zero, scale, X);
}

// ---- thick-restarted Arnoldi -----------------------------------------------------------------
// Upper Hessenberg form Z^T A Z of a dense m x m matrix (row-major, in
// place) with Z e_m = e_m: rows are reduced from the bottom up, row i by a
// Householder reflector on coordinates 0..i-1 that maps A[i, 0..i-1] to a
// multiple of e_{i-1}, so the last coordinate is never touched and the
// Arnoldi residual of a Ritz vector Z s keeps the form |h_{m+1,m}| |s_m|.
static void hessenberg_keep_last(std::vector<double>& A, int m, std::vector<double>& Z) {
  Z.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Z[(size_t)i * m + i] = 1.0;
  std::vector<double> v(m), tv;
  for (int i = m - 1; i >= 2; --i) {
    const int L = i;  // coordinates 0..L-1
    double nrm = 0.0;
    for (int j = 0; j < L; ++j) nrm += A[(size_t)i * m + j] * A[(size_t)i * m + j];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double xl = A[(size_t)i * m + L - 1];
    const double alpha = xl > 0 ? -nrm : nrm;
    for (int j = 0; j < L; ++j) v[j] = A[(size_t)i * m + j];
    v[L - 1] -= alpha;
    double vv = 0.0;
    for (int j = 0; j < L; ++j) vv += v[j] * v[j];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // A <- A H (columns 0..L-1 of every row), Z <- Z H
    for (std::vector<double>* M : {&A, &Z})
      for (int r = 0; r < m; ++r) {
        double* row = M->data() + (size_t)r * m;
        double t = 0.0;
        for (int j = 0; j < L; ++j) t += row[j] * v[j];
        t *= beta;
        for (int j = 0; j < L; ++j) row[j] -= t * v[j];
      }
    // A <- H A (rows 0..L-1): t = v^T A accumulated row by row (contiguous),
    // then the rank-one update
    tv.assign(m, 0.0);
    for (int j = 0; j < L; ++j) {
      const double* row = A.data() + (size_t)j * m;
      const double vj = v[j];
      for (int cc = 0; cc < m; ++cc) tv[cc] += vj * row[cc];
    }
    for (int j = 0; j < L; ++j) {
      double* row = A.data() + (size_t)j * m;
      const double bv = beta * v[j];
      for (int cc = 0; cc < m; ++cc) row[cc] -= bv * tv[cc];
    }
    for (int j = 0; j < L - 1; ++j) A[(size_t)i * m + j] = 0.0;
  }
}

// Leading eigenvalues by Arnoldi restarted thick (Morgan's restart with
// Ritz vectors, the same space as Krylov-Schur with exact shifts): after m
// steps the real and imaginary parts of the `keep` leading Ritz vectors
// (pairs whole), orthonormalized, become the first basis vectors, the last
// Arnoldi vector follows them, and the projected matrix restarts as their
// k x k block plus the residual row.  No filter and no locking: converged
// vectors stay in the kept set.  Workspace layout as the Chebyshev driver.
static int arnoldi_thick(kv_ctx* c, const kv_arnoldi_params* p, int sym_ref, int sym_rot, double* lam_re,
                         double* lam_im, double* resid, double* evecs, kv_eig_info* info) {
  const int64_t n = c->g.n;
  const int m = p->krylov_dim;
  int rc;
  double* V = c->ws;
  double* zp = V + (int64_t)(m + 1) * n;
  double* zc = zp + n;
  double* tmp = zc + n;
  double* L = tmp + n;
  double* Ys = L + (int64_t)(p->n_eigs + 1) * n;
  EigScope scope(c, sym_ref, sym_rot, L);
  // with a spectral transform the Krylov operator is C = (A - pole)^-1 (A - zero)
  // and the wanted values are its dominant ones
  struct StScope {
    kv_ctx* c;
    explicit StScope(kv_ctx* cc) : c(cc) {
      c->st_on = c->st_kind != KV_ST_NONE;
      c->st_inner = false;
      c->st_matvecs = 0;
      c->st_solves = 0;
    }
    ~StScope() {
      c->st_on = c->st_inner = false;
      c->pc_active = false;
    }
  } st_scope(c);
  const bool st = c->st_on;
  const int sel_order = st ? SEL_LARGEST : SEL_LEADING;
  auto eig_of = [&](std::complex<double> th) {
    return st ? (c->st_pole * th - c->st_zero) / (th - 1.0) : th;
  };
  auto eig_info = [&](int nout, int mv, int rs, int cv) {
    kv_eig_info e{nout, mv, rs, cv, c->relaxed_qr, 0};
    e.inner_matvecs = (int)std::min<long long>(c->st_matvecs, 2147483647LL);
    return e;
  };
  c->relaxed_qr = 0;
  HIPCHK(c, hipMemcpyAsync(V, p->v0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if ((rc = project_inplace(c, V))) return rc;
  if (sym_ref || sym_rot) HIPCHK(c, launch_symmetry_class(c, V, V, sym_ref, sym_rot));
  double vn = std::sqrt(std::max(0.0, dot1(c, V, V, &rc)));
  if (rc) return rc;
  if (!(vn > 0) || !std::isfinite(vn)) return fail(c, KV_ENONFINITE, "zero or non-finite start vector");
  if ((rc = lincomb(c, 1, {1.0 / vn}, {V}, V))) return rc;
  const char* ev = getenv("KV_ARNOLDI_TRACE");
  const bool trace = ev && atoi(ev) != 0;
  std::vector<double> H, A((size_t)m * m), Z, Hh;
  int matvecs = 0, restarts = 0, k0 = 0;
  bool conv = false;
  Ritz rz;
  std::vector<int> wsel;  // indices (into rz.sel order) of the wanted values
  for (;;) {
    int k = 0;
    if ((rc = arnoldi(c, V, m, H, &k, &matvecs, k0))) {
      if (info) *info = eig_info(0, matvecs, restarts, 0);
      return rc;
    }
    // Hessenberg form of the projected k x k matrix, last coordinate fixed
    const int ld = m + 1;
    A.assign((size_t)k * k, 0.0);
    for (int r = 0; r < k; ++r)
      for (int cc = 0; cc < k; ++cc) A[(size_t)r * k + cc] = H[r + (size_t)cc * ld];
    hessenberg_keep_last(A, k, Z);
    Hh.assign((size_t)ld * m, 0.0);
    for (int r = 0; r < k; ++r)
      for (int cc = std::max(0, r - 1); cc < k; ++cc) Hh[r + (size_t)cc * ld] = A[(size_t)r * k + cc];
    if (k < m || k == m) Hh[k + (size_t)(k - 1) * ld] = (k < m) ? 0.0 : H[m + (size_t)(m - 1) * ld];
    const int nkeep = std::min({p->keep, k - 2, 63});
    if ((rc = ritz(c, Hh, m, k, std::max(nkeep, p->n_eigs), rz, sel_order))) {
      if (info) *info = eig_info(0, matvecs, restarts, 0);
      return rc;
    }
    // the wanted set (first n_eigs in leading order, or of largest modulus
    // under a transform; a pair whole) inside rz.sel
    const std::vector<int> want = st ? modulus_set(rz.vals, p->n_eigs, true) : wanted_set(rz.vals, p->n_eigs);
    double scale = 0.0;
    for (int i : want) scale = std::max(scale, std::abs(rz.vals[i]));
    wsel.clear();
    bool all = true;
    for (int i : want) {
      const int q = (int)(std::find(rz.sel.begin(), rz.sel.end(), i) - rz.sel.begin());
      wsel.push_back(q);
      if (!(rz.res[q] <= p->tol * scale)) all = false;
    }
    conv = all || k < m;
    if (trace) {
      double rmx = 0.0;
      for (int q : wsel) rmx = std::max(rmx, rz.res[q]);
      fprintf(stderr, "[arnoldi-thick] restart %d matvecs %d res/scale %.3e", restarts, matvecs, rmx / scale);
      if (st) fprintf(stderr, " inner matvecs %lld", c->st_matvecs);
      for (size_t q = 0; q < wsel.size() && q < 4; ++q) {
        const auto lam = eig_of(rz.vals[rz.sel[wsel[q]]]);
        fprintf(stderr, "  (%.6g, %.6g)", lam.real(), lam.imag());
      }
      fprintf(stderr, "\n");
    }
    if (conv || matvecs + (m - nkeep) > p->max_matvec || (p->max_restarts > 0 && restarts >= p->max_restarts) ||
        p->max_restarts == 0)
      break;
    // kept set: the leading nkeep Ritz values of rz.sel (a pair whole), as
    // real coefficient vectors in the V basis (Z s), orthonormalized
    int kq = 0;
    std::vector<std::vector<double>> Wc;
    for (int q = 0; q < (int)rz.sel.size() && kq < nkeep; ++q) {
      const auto th = rz.vals[rz.sel[q]];
      if (th.imag() < 0) continue;  // its +Im partner carries the pair
      const int parts = th.imag() > 0 ? 2 : 1;
      if (kq + parts > 63) break;
      for (int part = 0; part < parts; ++part) {
        std::vector<double> w(k, 0.0);
        for (int r = 0; r < k; ++r) {
          double acc = 0.0;
          for (int t = 0; t < k; ++t)
            acc += Z[(size_t)r * k + t] * (part == 0 ? rz.vecs[q][t].real() : rz.vecs[q][t].imag());
          w[r] = acc;
        }
        // twice modified Gram-Schmidt against the kept ones
        for (int pass = 0; pass < 2; ++pass)
          for (const auto& u : Wc) {
            double d = 0.0;
            for (int r = 0; r < k; ++r) d += u[r] * w[r];
            for (int r = 0; r < k; ++r) w[r] -= d * u[r];
          }
        double nw = 0.0;
        for (double x : w) nw += x * x;
        nw = std::sqrt(nw);
        if (!(nw > 1e-12)) continue;  // dependent: drop
        for (double& x : w) x /= nw;
        Wc.push_back(w);
        ++kq;
      }
    }
    if (kq < 1) return fail(c, KV_ENOCONV, "thick restart: no Ritz vector kept");
    // T = W^T G W and the residual row h_{m+1,m} W[m-1, :]
    std::vector<double> GW((size_t)k * kq, 0.0);
    for (int cc = 0; cc < kq; ++cc)
      for (int r = 0; r < k; ++r) {
        double acc = 0.0;
        for (int t = 0; t < k; ++t) acc += H[r + (size_t)t * ld] * Wc[cc][t];
        GW[(size_t)r * kq + cc] = acc;
      }
    const double hlast = H[m + (size_t)(m - 1) * ld];
    std::vector<double> Hn((size_t)ld * m, 0.0);
    for (int r = 0; r < kq; ++r)
      for (int cc = 0; cc < kq; ++cc) {
        double acc = 0.0;
        for (int t = 0; t < k; ++t) acc += Wc[r][t] * GW[(size_t)t * kq + cc];
        Hn[r + (size_t)cc * ld] = acc;
      }
    for (int cc = 0; cc < kq; ++cc) Hn[kq + (size_t)cc * ld] = hlast * Wc[cc][k - 1];
    H.swap(Hn);
    // V[0..kq) = V W in place, then the last Arnoldi vector becomes V[kq]
    std::vector<double> Wrow((size_t)k * kq);
    for (int r = 0; r < k; ++r)
      for (int cc = 0; cc < kq; ++cc) Wrow[(size_t)r * kq + cc] = Wc[cc][r];
    double* dW = c->hess;  // the Hessenberg area is free between cycles
    if ((rc = upload(c, dW, Wrow.data(), Wrow.size() * sizeof(double)))) return rc;
    HIPCHK(c, launch_combine(c, V, n, k, dW, kq, V, n));
    HIPCHK(c, hipMemcpyAsync(V + (int64_t)kq * n, V + (int64_t)m * n, n * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    // back into range(P) (and the class): A = P J has the eigenvalue 0 on
    // gradient fields, right of every wanted value of a stable state, and
    // the restarts amplify the round-off the basis carries there until a
    // spurious Ritz value 0 converges (seen on the Gr = 0 conduction state)
    for (int q = 0; q <= kq; ++q) {
      double* vq = V + (int64_t)q * n;
      if ((rc = project_inplace(c, vq))) return rc;
      if (sym_ref || sym_rot) HIPCHK(c, launch_symmetry_class(c, vq, vq, sym_ref, sym_rot));
    }
    k0 = kq;
    ++restarts;
  }
  // outputs: the wanted values of A in leading order.  Under the transform
  // lambda = (pole theta - zero) / (theta - 1) and Im theta = (zero - pole)
  // Im lambda / |lambda - pole|^2, so the +Im member of a pair of A is the
  // -Im member of C; its Ritz vector is the eigenvector of both
  const int nout = (int)wsel.size();
  std::vector<std::complex<double>> lam(nout);
  std::vector<int> ord(nout);
  for (int q = 0; q < nout; ++q) {
    lam[q] = eig_of(rz.vals[rz.sel[wsel[q]]]);
    ord[q] = q;
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (lam[a].real() != lam[b].real()) return lam[a].real() > lam[b].real();
    return lam[a].imag() > lam[b].imag();
  });
  for (int r = 0; r < nout; ++r) {
    lam_re[r] = lam[ord[r]].real();
    lam_im[r] = lam[ord[r]].imag();
    if (resid) resid[r] = rz.res[wsel[ord[r]]];
  }
  if (evecs) {
    // Ritz vectors V Z s of the wanted values (real and imaginary parts) into
    // the Ritz slots, then normalized and turned like the Chebyshev driver's
    const int k = (int)rz.vecs.empty() ? 0 : (int)rz.vecs[0].size();
    std::vector<const double*> src_re(nout, nullptr), src_im(nout, nullptr);
    std::vector<int> nl(nout, 0), outidx(nout);
    std::vector<std::complex<double>> vals(nout);
    int slot = 0;
    for (int r = 0; r < nout; ++r) {
      const int q = ord[r];
      vals[r] = lam[q];
      outidx[r] = r;
      if (lam[q].imag() < 0) {
        src_re[r] = src_re[r - 1];
        src_im[r] = src_im[r - 1];
        continue;
      }
      const int parts = lam[q].imag() > 0 ? 2 : 1;
      std::vector<double> Wrow((size_t)k * parts);
      for (int rr = 0; rr < k; ++rr)
        for (int part = 0; part < parts; ++part) {
          double acc = 0.0;
          for (int t = 0; t < k; ++t)
            acc += Z[(size_t)rr * k + t] *
                   (part == 0 ? rz.vecs[wsel[q]][t].real() : rz.vecs[wsel[q]][t].imag());
          Wrow[(size_t)rr * parts + part] = acc;
        }
      if (slot + parts > p->n_eigs + 1) return fail(c, KV_EINVAL, "eigenvector workspace exhausted");
      if ((rc = upload(c, c->hess, Wrow.data(), Wrow.size() * sizeof(double)))) return rc;
      HIPCHK(c, launch_combine(c, V, n, k, c->hess, parts, Ys + (int64_t)slot * n, n));
      src_re[r] = Ys + (int64_t)slot * n;
      src_im[r] = parts == 2 ? src_re[r] + n : nullptr;
      slot += parts;
    }
    c->nlock = 0;
    if ((rc = write_eigenvectors(c, L, outidx, vals, src_re, src_im, nl, evecs, zp, zc, tmp, &matvecs))) return rc;
  }
  if (info) *info = eig_info(nout, matvecs, restarts, conv ? 1 : 0);
  if (!conv && p->max_restarts > 0) return fail(c, KV_ENOCONV, "Arnoldi: not converged within the budget");
  return KV_OK;
}

// ---- Chebyshev-preconditioned Arnoldi -------------------------------------------------------
int kv_arnoldi_leading_eigs(kv_ctx* c, const kv_arnoldi_params* p, double* lam_re, double* lam_im,
                            double* resid, double* evecs, kv_eig_info* info) {
  if (!c) return KV_EINVAL;
  if (!p || !lam_re || !lam_im || !p->v0) return fail(c, KV_EINVAL, "null argument");
  int sym_ref = 0, sym_rot = 0, rc;
  if ((rc = check_sym(c, p->flags, &sym_ref, &sym_rot))) return rc;
  const int m = p->krylov_dim;
  if (m < 2 || m > 400 || p->n_eigs < 1 || p->n_eigs >= m || p->max_matvec < m || p->max_restarts < 0)
    return fail(c, KV_EINVAL, "bad Arnoldi parameters");
  if (!c->has_base) return fail(c, KV_ESTATE, "no base flow");
  const int64_t n = c->g.n;
  if ((rc = check_finite(c, p->v0, n, "v0"))) return rc;
  MixedScope mixed(c);
  // workspace: V (m+1 vectors) + z_prev, z, tmp + up to n_eigs+1 locked
  // vectors (+ as many lock-time Ritz vectors when eigenvectors are asked for)
  const int nslot = p->n_eigs + 1;
  if ((rc = ws_bind(c, KV_WS_ARNOLDI, m, p->n_eigs))) return rc;
  if (p->keep > 0) {
    if (p->keep <= p->n_eigs || p->keep > m - 2) return fail(c, KV_EINVAL, "keep must be in n_eigs+1..krylov_dim-2");
    return arnoldi_thick(c, p, sym_ref, sym_rot, lam_re, lam_im, resid, evecs, info);
  }
  if (c->st_kind != KV_ST_NONE) return fail(c, KV_EINVAL, "a spectral transform needs the thick restart (keep > 0)");
  double* V = c->ws;
  double* zp = c->ws + (int64_t)(m + 1) * n;
  double* zc = zp + n;
  double* tmp = zc + n;
  double* L = tmp + n;
  double* Ys = L + (int64_t)nslot * n;  // lock-time Ritz vectors (real, imaginary part), if evecs
  int nys = 0;
  EigScope scope(c, sym_ref, sym_rot, L);
  c->relaxed_qr = 0;
  // the start vector in range(P), in the class, W-orthogonal to the locked vectors
  auto settle = [&](double* v) -> int {
    int r;
    if ((r = project_inplace(c, v))) return r;
    if (sym_ref || sym_rot) HIPCHK(c, launch_symmetry_class(c, v, v, sym_ref, sym_rot));
    return deflate(c, v);
  };
  HIPCHK(c, hipMemcpyAsync(V, p->v0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if ((rc = settle(V))) return rc;
  int matvecs = 0, restarts = 0;
  std::vector<double> H;
  Ritz rz;
  bool conv = false;
  // output values (locked, then the last cycle's wanted ones), their residual
  // estimates, where their Ritz vector is (Ys slot of its real part, or -1:
  // the last cycle's basis, entry lk_q of the Ritz data) and how many locked
  // vectors were deflated when it was found
  std::vector<std::complex<double>> lk_vals;
  std::vector<double> lk_res;
  std::vector<int> lk_slot, lk_q, lk_nl;
  // KV_ARNOLDI_TRACE=1: one line per restart on stderr (residual, ellipse,
  // filter degree, wanted Ritz values, locked count)
  const char* ev = getenv("KV_ARNOLDI_TRACE");
  const bool trace = ev && atoi(ev) != 0;
  for (;;) {
    double vn = std::sqrt(std::max(0.0, dot1(c, V, V, &rc)));
    if (rc) return rc;
    if (!(vn > 0) || !std::isfinite(vn)) return fail(c, KV_ENONFINITE, "zero or non-finite start vector");
    if ((rc = lincomb(c, 1, {1.0 / vn}, {V}, V))) return rc;
    int k = 0;
    if ((rc = arnoldi(c, V, m, H, &k, &matvecs)) ||
        (rc = ritz(c, H, m, k, p->n_eigs - (int)lk_vals.size(), rz))) {
      if (info) *info = kv_eig_info{0, matvecs, restarts, 0, c->relaxed_qr};  // the work done so far
      return rc;
    }
    double scale = 0.0;
    for (int i : rz.sel) scale = std::max(scale, std::abs(rz.vals[i]));
    for (const auto& v : lk_vals) scale = std::max(scale, std::abs(v));
    // converged prefix of the wanted set in leading order; a pair stays whole
    // (its members' residual estimates agree to round-off)
    size_t ndone = 0;
    while (ndone < rz.sel.size() && rz.res[ndone] <= p->tol * scale) ++ndone;
    if (ndone > 0 && ndone < rz.sel.size() && rz.vals[rz.sel[ndone - 1]].imag() > 0 &&
        std::abs(rz.vals[rz.sel[ndone]] - std::conj(rz.vals[rz.sel[ndone - 1]])) <=
            1e-12 * std::max(1.0, std::abs(rz.vals[rz.sel[ndone - 1]])))
      ++ndone;
    conv = ndone == rz.sel.size() || k < m;  // k < m: invariant subspace found
    const bool stop = conv || matvecs >= p->max_matvec || restarts >= p->max_restarts;
    // lock: converged values (or, at the end, all wanted ones) join the output;
    // before a restart their real invariant subspaces join L
    const size_t nout = stop ? rz.sel.size() : ndone;
    for (size_t q = 0; q < nout; ++q) {
      const bool minus = rz.vals[rz.sel[q]].imag() < 0;
      lk_vals.push_back(rz.vals[rz.sel[q]]);
      lk_res.push_back(rz.res[q]);
      lk_q.push_back((int)q);
      lk_nl.push_back(minus && !lk_nl.empty() ? lk_nl.back() : c->nlock);
      lk_slot.push_back(stop ? -1 : (minus && !lk_slot.empty() ? lk_slot.back() : (evecs ? nys : -1)));
      if (stop || minus) continue;  // a pair locks once, by its +Im member
      const int parts = rz.vals[rz.sel[q]].imag() > 0 ? 2 : 1;
      for (int part = 0; part < parts; ++part) {
        double* dst = L + (int64_t)c->nlock * n;
        double* ys = evecs ? Ys + (int64_t)(nys + part) * n : dst;
        std::vector<double> coef(k);
        for (int r = 0; r < k; ++r) coef[r] = -(part == 0 ? rz.vecs[q][r].real() : rz.vecs[q][r].imag());
        HIPCHK(c, launch_fill(c, n, 0.0, ys));
        if ((rc = upload(c, c->dres, coef.data(), k * sizeof(double)))) return rc;
        HIPCHK(c, launch_mupdate(c, V, n, k, c->dres, ys));
        if (ys != dst) HIPCHK(c, hipMemcpyAsync(dst, ys, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if ((rc = deflate(c, dst))) return rc;
        const double ln = std::sqrt(std::max(0.0, dot1(c, dst, dst, &rc)));
        if (rc) return rc;
        if (!(ln > 0) || !std::isfinite(ln)) return fail(c, KV_ENONFINITE, "degenerate locked vector");
        if ((rc = lincomb(c, 1, {1.0 / ln}, {dst}, dst))) return rc;
        ++c->nlock;
      }
      if (evecs) nys += parts;
    }
    if (stop) break;
    if ((int)lk_vals.size() >= p->n_eigs) {  // every wanted value locked
      conv = true;
      break;
    }
    // the wanted values still open
    std::vector<int> rest(rz.sel.begin() + ndone, rz.sel.end());
    // filter: an ellipse around the unwanted Ritz values and a degree
    std::vector<std::complex<double>> unw;
    for (int i = 0; i < k; ++i)
      if (std::find(rz.sel.begin(), rz.sel.end(), i) == rz.sel.end()) unw.push_back(rz.vals[i]);
    int deg = 0;
    double d = 0, a = 0, bb = 0, c2 = 0, wr = 0;
    if (!unw.empty()) {
      double ref = 1e300;
      for (int i : rest) ref = std::min(ref, rz.vals[i].real());
      ellipse(unw, ref, &d, &a, &bb, &c2);
      wr = ref - d;
      deg = cheb_degree(wr, a, bb, c2, p->cheb_degree_max);
      deg = std::min(deg, std::max(0, p->max_matvec - matvecs - m));
    }
    // restart vector: sum of the real and imaginary parts of the open wanted
    // Ritz vectors, each weighted by the inverse of its growth under the
    // filter, growth_rate(lambda - d)^deg, relative to the least growing one;
    // unweighted, a value far right of the ellipse outgrows the others by
    // many orders and they sink to round-off in the filtered vector
    std::vector<double> wts(rest.size(), 1.0);
    if (deg > 0) {
      std::vector<double> lg(rest.size());
      double lmin = 1e300;
      for (size_t q = 0; q < rest.size(); ++q) {
        lg[q] = deg * std::log(growth_rate(rz.vals[rest[q]] - d, a, bb, c2));
        lmin = std::min(lmin, lg[q]);
      }
      for (size_t q = 0; q < rest.size(); ++q) wts[q] = std::max(std::exp(lmin - lg[q]), 1e-300);
    }
    std::vector<double> coef(k, 0.0);
    for (size_t q = 0; q < rest.size(); ++q)
      for (int r = 0; r < k; ++r)
        coef[r] += wts[q] * (rz.vecs[ndone + q][r].real() + rz.vecs[ndone + q][r].imag());
    for (int r = 0; r < k; ++r) coef[r] = -coef[r];
    HIPCHK(c, launch_fill(c, n, 0.0, zc));
    if ((rc = upload(c, c->dres, coef.data(), k * sizeof(double)))) return rc;
    HIPCHK(c, launch_mupdate(c, V, n, k, c->dres, zc));
    if ((rc = deflate(c, zc))) return rc;
    double zn = std::sqrt(std::max(0.0, dot1(c, zc, zc, &rc)));
    if (rc) return rc;
    if ((rc = lincomb(c, 1, {1.0 / zn}, {zc}, zc))) return rc;
    if (trace) {
      double rmx = 0.0;
      for (double r : rz.res) rmx = std::max(rmx, r);
      fprintf(stderr, "[arnoldi] restart %d matvecs %d res/scale %.3e  ellipse d %.4g a %.4g b %.4g  degree %d  locked %d",
              restarts, matvecs, rmx / scale, d, a, bb, deg, (int)lk_vals.size());
      for (size_t q = 0; q < rz.sel.size() && q < 4; ++q)
        fprintf(stderr, "  (%.6g, %.6g)", rz.vals[rz.sel[q]].real(), rz.vals[rz.sel[q]].imag());
      fprintf(stderr, "\n");
    }
    if (deg > 0) {
      // z1 = r1 (A - d) z0, z_{j+1} = r_{j+1} (2 (A - d) z_j - c^2 r_j z_{j-1}),
      // A deflated by the locked vectors (inside matvec)
      double rj = 1.0 / wr;
      HIPCHK(c, hipMemcpyAsync(zp, zc, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      if ((rc = matvec(c, zp, tmp))) return rc;
      ++matvecs;
      if ((rc = lincomb(c, 2, {rj, -d * rj}, {tmp, zp}, zc))) return rc;
      for (int it = 1; it < deg; ++it) {
        const double rn = 1.0 / (2.0 * wr - c2 * rj);
        if ((rc = matvec(c, zc, tmp))) return rc;
        ++matvecs;
        // new = rn * (2 tmp - 2 d zc - c2 rj zp), stored in zp, then swap
        if ((rc = lincomb(c, 3, {2.0 * rn, -2.0 * d * rn, -c2 * rj * rn}, {tmp, zc, zp}, zp))) return rc;
        std::swap(zp, zc);
        rj = rn;
      }
    }
    // back into range(P): the filter's -d z term carries round-off onto gradient
    // fields, where A has the eigenvalue 0 (right of the wanted set)
    HIPCHK(c, hipMemcpyAsync(V, zc, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if ((rc = settle(V))) return rc;
    ++restarts;
  }
  // the n_eigs leading of the locked values (a pair kept whole)
  const std::vector<int> out = wanted_set(lk_vals, p->n_eigs);
  for (size_t q = 0; q < out.size(); ++q) {
    lam_re[q] = lk_vals[out[q]].real();
    lam_im[q] = lk_vals[out[q]].imag();
    if (resid) resid[q] = lk_res[out[q]];
  }
  if (evecs) {
    std::vector<const double*> src_re(out.size(), nullptr), src_im(out.size(), nullptr);
    std::vector<int> nl(out.size(), 0);
    // the last cycle's Ritz vectors, still in V, go to the Ys slots left free
    for (size_t q = 0; q < out.size(); ++q) {
      const int e = out[q];
      nl[q] = lk_nl[e];
      if (lk_slot[e] < 0 && lk_vals[e].imag() >= 0) {
        const int parts = lk_vals[e].imag() > 0 ? 2 : 1;
        if (nys + parts > nslot) return fail(c, KV_EINVAL, "eigenvector workspace exhausted");
        for (int part = 0; part < parts; ++part) {
          double* ys = Ys + (int64_t)(nys + part) * n;
          std::vector<double> coef(rz.vecs[lk_q[e]].size());
          for (size_t r = 0; r < coef.size(); ++r)
            coef[r] = -(part == 0 ? rz.vecs[lk_q[e]][r].real() : rz.vecs[lk_q[e]][r].imag());
          HIPCHK(c, launch_fill(c, n, 0.0, ys));
          if ((rc = upload(c, c->dres, coef.data(), coef.size() * sizeof(double)))) return rc;
          HIPCHK(c, launch_mupdate(c, V, n, (int)coef.size(), c->dres, ys));
        }
        lk_slot[e] = nys;
        nys += parts;
      } else if (lk_slot[e] < 0) {
        lk_slot[e] = lk_slot[out[q - 1]];  // the -Im member follows its +Im member
      }
      src_re[q] = Ys + (int64_t)lk_slot[e] * n;
      src_im[q] = lk_vals[e].imag() != 0.0 ? src_re[q] + n : nullptr;
    }
    if ((rc = write_eigenvectors(c, L, out, lk_vals, src_re, src_im, nl, evecs, zp, zc, tmp, &matvecs))) return rc;
  }
  if (info) *info = kv_eig_info{(int)out.size(), matvecs, restarts, conv ? 1 : 0, c->relaxed_qr};
  if (!conv && p->max_restarts > 0) return fail(c, KV_ENOCONV, "Arnoldi: not converged within the budget");
  return KV_OK;
}

int kv_hessenberg_eigenvalues(kv_ctx* c, const double* H, int m, double* wr, double* wi) {
  if (!c) return KV_EINVAL;
  if (!H || !wr || !wi) return fail(c, KV_EINVAL, "null argument");
  if (m < 1 || m > 400) return fail(c, KV_EINVAL, "m must be in 1..400");
  std::vector<double> Hk((size_t)m * m, 0.0);
  for (int r = 0; r < m; ++r)
    for (int cc = std::max(0, r - 1); cc < m; ++cc) {
      const double v = H[(size_t)r * m + cc];
      if (!std::isfinite(v)) return fail(c, KV_ENONFINITE, "non-finite Hessenberg entry");
      Hk[(size_t)r * m + cc] = v;
    }
  int rc;
  const size_t mm = (size_t)m * m;
  double *dH = c->hess_small, *dwr = dH + mm, *dwi = dwr + m;  // (400^2 + 2 400 + 2) doubles
  int* dinfo = reinterpret_cast<int*>(dwi + m);
  if ((rc = upload(c, dH, Hk.data(), mm * sizeof(double)))) return rc;
  HIPCHK(c, launch_hessenberg_values(c->stream, dH, m, dwr, dwi, dinfo));
  int info = 0;
  HIPCHK(c, hipMemcpyAsync(wr, dwr, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(wi, dwi, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info & 1) return fail(c, KV_ENOCONV, "Hessenberg QR did not converge");
  return KV_OK;
}

int kv_timing(kv_ctx* c, int enable, double ms[4], int calls[2]) {
  if (!c) return KV_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double acc[4] = {0, 0, 0, 0};
  int cnt[4] = {0, 0, 0, 0};
  for (auto& m : c->ev_marks) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, m.second.first, m.second.second) == hipSuccess) {
      acc[m.first] += t;
      cnt[m.first] += 1;
    }
    c->ev_pool.push_back(m.second.first);
    c->ev_pool.push_back(m.second.second);
  }
  c->ev_marks.clear();
  if (ms)
    for (int q = 0; q < 4; ++q) ms[q] = acc[q];
  if (calls) {
    calls[0] = cnt[0];
    calls[1] = cnt[2];
  }
  c->timing = enable != 0;
  return KV_OK;
}

const char* kv_last_error(const kv_ctx* c) { return c ? c->err.c_str() : kNoCtx; }

}  // extern "C"
