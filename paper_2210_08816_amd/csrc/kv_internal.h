// Internal declarations of the gfx950 Krylov-vector library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kv.h"

namespace kv {

// Per-axis metrics on the device.  n cells, faces 0..n.
//   h[i]    cell width, i < n           ih[i] = 1/h[i]
//   id[f]   1/(centre gap) at face f, f = 0..n; the wall gaps are h/2
//   wlo[f], whi[f]  interpolation weights of cells f-1 and f at interior face f
//   sq[i]   sqrt(h[i])                  isq[i] = 1/sqrt(h[i])
//   dd[f]   centre gap at face f (control-volume width of a face unknown)
//   lam[i]  eigenvalues of the symmetric 1-D Neumann operator (FD basis)
//   c[i]    cell-centre coordinate
struct Axis {
  int n;
  const double *h, *ih, *id, *wlo, *whi, *sq, *isq, *dd, *lam, *c;
};

// One 1-D operator H^-1 K of the Stokes/heat preconditioner (H diagonal
// widths, K symmetric positive (semi)definite): M = H^-1/2 K H^-1/2 =
// Q diag(lam) Q^T, with s = H^1/2 folded into the transform matrices
// (row-major n x n):  fwdB = diag(s) Q (x pass), fwdA = Q^T diag(s) (y, z
// passes), invB = Q^T diag(1/s), invA = diag(1/s) Q.
struct HelmBasis {
  int n = 0;
  const double *fwdB = nullptr, *fwdA = nullptr, *invB = nullptr, *invA = nullptr, *lam = nullptr;
};
enum { HB_CN = 0, HB_CD = 1, HB_FD = 2 };  // centre Neumann, centre Dirichlet, face Dirichlet

// Everything a stencil or vector kernel needs about the grid and the layout.
struct Grid {
  int nx, ny, nz;
  int64_t ou, ov, ow, oT, n;  // packed offsets and size
  Axis ax[3];
  double nu, kappa, beta;
  int null3;                  // flat index (c*ny + b)*nx + a of the FD null mode
};

}  // namespace kv

struct kv_ctx {
  kv::Grid g;
  int64_t ncell = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  double Gr = 0, Pr = 0;
  // host copies of the metrics (used by host-side solver bookkeeping)
  std::vector<double> hf[3];
  // device allocations
  double* metric = nullptr;   // all Axis arrays
  double* Qf[3] = {nullptr, nullptr, nullptr};   // Q (n x n row-major): forward uses Q
  double* Qt[3] = {nullptr, nullptr, nullptr};   // Q^T
  int split[3] = {0, 0, 0};   // 1: mirror-symmetric axis, Qf/Qt hold the even/odd half bases
  float* Qf32[3] = {nullptr, nullptr, nullptr};  // FP32 copies of the split bases (mixed form)
  float* Qt32[3] = {nullptr, nullptr, nullptr};
  double* ymix = nullptr;     // FP64 scratch vector of the mixed refinement sweeps (in the workspace)
  double* cell_part = nullptr;  // per-block maxima of the cell-grid kernels (2 per block)
  int64_t cell_part_len = 0;
  double* X0 = nullptr;       // base flow copy
  bool has_base = false;
  double* cellA = nullptr;    // two cell-sized scratch fields for the Poisson solve
  double* cellB = nullptr;
  double* part = nullptr;     // reduction partials
  double* dres = nullptr;     // reduction results on the device (64 doubles)
  double* hres = nullptr;     // pinned host mirror of dres
  double* dcoef = nullptr;    // device coefficients of the Gram-Schmidt updates (1024 doubles)
  double* hcoef = nullptr;    // pinned host staging of dcoef
  int npart_blocks = 0;
  int nmd_blocks = 0;         // blocks of the multi-dot kernels (their partials also in part)
  // caller-owned workspace (kv_set_workspace): solver vectors, Krylov
  // bases, the mixed-form scratch vector and the Ritz-vector work area are
  // carved from it per call; the library never allocates them
  double* ws = nullptr;
  size_t ws_bytes = 0;
  double* hess = nullptr;     // Hessenberg / Ritz-vector area inside the workspace (Arnoldi)
  double* hess_small = nullptr;  // owned: kv_hessenberg_eigenvalues, m <= 400
  void* xfer = nullptr;       // owned: interpolation tables of kv_state_from_cells
  size_t xfer_bytes = 0;
  // Stokes/heat preconditioner (kv_set_preconditioner)
  kv::HelmBasis hb[3][3];     // [axis][HB_*]
  double* pc_mem = nullptr;   // device storage of all bases
  // workspace vectors of a preconditioned call:
  double* pc_tmp = nullptr;   // M^-1 x inside the preconditioned operator
  double* pc_d0 = nullptr;    // copy of the caller's initial iterate
  double* pc_scr = nullptr;   // intermediate passes of the Helmholtz solves
  int pc_kind = 0;            // KV_PC_NONE or KV_PC_STOKES
  double pc_sigma = 0.0;
  bool pc_active = false;     // set while a preconditioned solve runs
  int gmres_m = 40;           // restart length of the GMRES continuation of the Newton correction
  int stall_cycles = 50;      // BiCGstab(2) cycles without a 10% residual drop before GMRES takes over
  int gmres_defl = 0;         // harmonic Ritz vectors kept across GMRES restarts (0: plain restarts)
  int sym_ref = 0, sym_rot = 0;  // symmetry class kept by matvec while a restricted Arnoldi runs
  const double* lockQ = nullptr;  // locked W-orthonormal vectors matvec deflates while Arnoldi runs
  int nlock = 0;
  int relaxed_qr = 0;         // Arnoldi cycles whose Hessenberg QR deflated by the relaxed test
  // spectral transform of Arnoldi (kv_set_spectral_transform): Cayley
  // C = (A - pole)^-1 (A - zero), the inverse by preconditioned GMRES
  int st_kind = 0;            // KV_ST_NONE or KV_ST_CAYLEY
  double st_pole = 0.0, st_zero = 0.0, st_tol = 1e-10;
  int st_max_matvec = 20000;  // budget of one inner solve
  bool st_on = false;         // set while a transformed Arnoldi runs
  bool st_inner = false;      // set while its inner solve runs: the operator is (A - pole) M^-1
  double* st_t = nullptr;     // workspace: the inner iterate
  double* st_V = nullptr;     // workspace: the inner GMRES basis (gmres_m + 1 vectors)
  long long st_matvecs = 0;   // applications of P J by the inner solves of one Arnoldi call
  int st_solves = 0;
  // projection of the solvers' operators (kv_set_solver_projection): the
  // mixed form while a Newton correction or an Arnoldi call runs
  bool solve_mixed_set = false;
  bool solve_mixed = false;
  double* ymix_solve = nullptr;  // workspace: the mixed sweeps' scratch vector
  // phase timing (kv_timing): events recorded around each phase while enabled
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;       // reusable events
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;  // (phase, start, stop)
  std::string err;
};

namespace kv {

// ---- launchers (all enqueue on ctx->stream) -----------------------------------
// y = J(X0) x (mode 0) or y = N(x) (mode 1, X0 unused), unprojected.
hipError_t launch_operator(const kv_ctx* c, const double* X0, const double* x, double* y, int mode);
// cellA = V^1/2 D y  (net face flux over sqrt of the cell volume)
hipError_t launch_scaled_divergence(const kv_ctx* c, const double* y, double* out);
// Whether the tiled stencil can write the scaled divergence of its output
// (the grid fits its 32-bit offsets and its LDS request is granted).
bool operator_fuses_divergence(const kv_ctx* c);
// y = J(X0) x, and div = V^1/2 D y except on the tiles' edge cells, which
// hold the partial unscaled net flux until launch_divergence_edges completes
// them (hipErrorNotSupported where the stencil cannot fuse).
hipError_t launch_operator_divergence(const kv_ctx* c, const double* X0, const double* x, double* y, double* div);
hipError_t launch_divergence_edges(const kv_ctx* c, const double* y, double* div);
// p = L^+ (V^-1/2 in) by fast diagonalization; in and out are cell fields.
// in is overwritten (used as scratch); result in out.
hipError_t launch_fd_solve(const kv_ctx* c, double* in, double* out);
// One axis pass of the even/odd split transform (mirror-symmetric axes).
hipError_t launch_fd_split_pass(const kv_ctx* c, int axis, bool inverse, int epi, const double* in, double* out);
hipError_t launch_fd_split_pass_f32(const kv_ctx* c, int axis, bool inverse, int epi, const float* in, float* out);
// FP32-storage Poisson solve (all axes split): in = scaled divergence, out = p
hipError_t launch_fd_solve_f32(const kv_ctx* c, float* in, float* out);
// The same with bf16x3 split products on the bf16 matrix cores
hipError_t launch_fd_solve_bf3(const kv_ctx* c, float* in, float* out);
// mixed form: FP32 b = V^1/2 D y from FP64 y
hipError_t launch_scaled_divergence_f32(const kv_ctx* c, const double* y, float* out);
// mixed form: yout = yin - G p (FP32 p), and from the corrected field the
// next scaled divergence bnext (FP32, may be null) and block maxima of
// |net flux| and |face flux| (c->part) finished into c->dres[0..2)
hipError_t launch_correct_divergence(kv_ctx* c, const double* yin, const float* p, double* yout, float* bnext);
// y_vel -= G p
hipError_t launch_gradient_correction(const kv_ctx* c, const double* p, double* y);

// Weighted dot products over the packed layout.  npair <= 4 pairs (a_i, b_i);
// results land in c->dres[0..npair).
hipError_t launch_wdots(kv_ctx* c, int npair, const double* const* a, const double* const* b,
                        double* out = nullptr);
// res[i] = <V_i, w>_W for i < nvec (V row stride ldv), results in out (device,
// default c->dres; nvec <= 512)
hipError_t launch_mdot(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* w, double* out = nullptr);
// out1[i] = <V_i, x1>_W, out2[i] = <V_i, x2>_W for i < nvec <= 512, one pass
// over V (device outputs)
hipError_t launch_mdot2(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* x1, const double* x2,
                       double* out1, double* out2);
// w <- cw w - cv v - sum_i d[i] V_i and v <- cn (v - sum_i sv[i] V_i), one
// pass over V (d, sv on the device, nvec <= 512 values, nvec may be 0)
hipError_t launch_mupdate2(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* d, const double* sv,
                           double cw, double cv, double cn, double* w, double* v);
// w -= sum_i h[i] V_i, h on the device (nvec values)
hipError_t launch_mupdate(kv_ctx* c, const double* V, int64_t ldv, int nvec, const double* h, double* w);
// out_q = sum_{j<m} W[j kq + q] V_j (V row stride ldv, out row stride ldo,
// W on the device, kq <= 64); out may be V itself with ldo == ldv
hipError_t launch_combine(const kv_ctx* c, const double* V, int64_t ldv, int m, const double* W, int kq,
                          double* out, int64_t ldo);
// out = sum_k coef[k] * in[k], k < nterm <= 4 (out may alias in[k])
hipError_t launch_lincomb(const kv_ctx* c, int64_t n, int nterm, const double* coef,
                          const double* const* in, double* out);
// out[0..n) = v
hipError_t launch_fill(const kv_ctx* c, int64_t n, double v, double* out);
// maxima: dres[0] = max|a| (or a NaN flag), used for non-finite checks and norms
hipError_t launch_maxabs(kv_ctx* c, const double* a, int64_t n);
// dres[0] = max |net flux|, dres[1] = max |face flux| of the velocity block of y
hipError_t launch_div_measure(kv_ctx* c, const double* y);
// dres[0..3) = R_ref, R_2D, R_3D of X
hipError_t launch_symmetry(kv_ctx* c, const double* X);
// y = projection of x onto a symmetry class; e_ref, e_rot in {-1, 0, +1}; y may equal x
hipError_t launch_symmetry_class(kv_ctx* c, const double* x, double* y, int e_ref, int e_rot);

// The mixed-form projection of y (kv_project with KV_MIXED) with its
// scratch vector ymix (n doubles) supplied by the caller.
int project_mixed_with(kv_ctx* c, double* y, double* div_out, int* sweeps_out, double* ymix);
bool mixed_grid(const kv_ctx* c);
// Bytes of device scratch the mixed projection needs on c's grid.
size_t mixed_scratch_bytes(const kv_ctx* c);
// Set-up of the library's static device scratch on the current device
// (kv_static.hip); called by kv_create.
int static_scratch_init(int device);

// FD GEMM self-test entry (C = A B, row-major), used by the unit test only.
// KV_FD_TILE=64 or 32: the tile shape every FD and Helmholtz GEMM pass must
// use (0: chosen from the sizes); read at each launch.
int fd_forced_tile();

// (sigma - coef (A_x + A_y + A_z))^-1 with A_a = -H_a^-1 K_a of the given
// bases, on a (bz.n, by.n, bx.n) block; 6 GEMM passes with cellA/cellB as
// scratch.  in may equal out.
hipError_t launch_fd_helmholtz4(const kv_ctx* c, const HelmBasis* const bx[4], const HelmBasis* const by[4],
                                const HelmBasis* const bz[4], double sigma, const double coef[4],
                                const double* const in[4], double* const out[4], double* const scr[4]);

// Network-grid transfers (kv_transfer.hip).  cells_from_state: out[c][K][J][I]
// = (volume average over the f^3 fine cells of the centre value - shift[c]) / scale[c].
hipError_t launch_cells_from_state(const kv_ctx* c, const double* X, int f, const double shift[4],
                                   const double scale[4], float* out);
// state_from_cells: trilinear interpolation on the extended network nodes;
// q/t: per axis the face table then the centre table (axis-major, 6 each).
// cells_ref non-null: X += interp(cells) - interp(cells_ref).
hipError_t launch_state_from_cells(const kv_ctx* c, const float* cells, const float* cells_ref, const int r[3],
                                   const int* const q[6], const double* const t[6], const double shift[4],
                                   const double scale[4], double* X);

// Hessenberg eigen-solve on the device: H (m x m, row-major, leading dim ld)
// -> eigenvalues (wr, wi) and, for the requested columns, eigenvector
// coefficients.  See kv_hess.hip.
hipError_t launch_hessenberg_eig(const kv_ctx* c, double* H, int m, int ld, double* Z, double* wr,
                                 double* wi, int* info, double* vr, double* vi, int want_vectors);

// Host symmetric eigen-solver (cyclic Jacobi) for the FD bases.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& lam);

}  // namespace kv
