/*
 * kv.h -- C ABI of the MI355X Krylov-vector library for Boussinesq convection
 * in a laterally heated cube (Gelfgat, "Sequence of bifurcations of natural
 * convection of air in a laterally heated cube with perfectly insulated
 * horizontal and spanwise boundaries").
 *
 * The library computes, on one gfx950 GPU, the hot path of the paper's
 * Newton / Arnoldi linear-stability method (Sec. 1 and Sec. 3): divergence-free
 * Krylov vectors y = P J(X0) x that satisfy all boundary conditions, the
 * steady residual F = P N(X), Newton corrections by BiCGstab(2) combined with
 * GMRES, and leading eigenvalues by Chebyshev-preconditioned Arnoldi
 * iteration without shift-and-invert.
 *
 * Equations (Sec. 2, Eqs. 1-3, the paper's scaling): nu = Gr^-1/2,
 * kappa = 1/(Pr Gr^1/2), buoyancy +T e_z; no-slip walls, T = 1 / 0 on x = 0 / 1
 * (Eq. 4), adiabatic y- and z-walls (Eqs. 5-6).  Gr == 0 selects the viscous
 * scaling nu = 1, kappa = 1/Pr, no buoyancy.
 *
 * Discretization: second-order conservative staggered (MAC) finite volumes on
 * a tensor-product grid of the unit cube, cell centres at face midpoints,
 * distance-linear centre-to-face interpolation, wall values at half-cell
 * distance.  The pressure is not a state variable: P = I - G (D G)^+ D is the
 * discrete Leray projection, applied by fast diagonalization (exact in one
 * pass in FP64).
 *
 * Packed state vector (all vector arguments): FP64, x fastest, then y, then z,
 *   [ u: (nz, ny, nx-1) | v: (nz, ny-1, nx) | w: (nz-1, ny, nx) | T: (nz, ny, nx) ]
 * u on interior x-faces, v on interior y-faces, w on interior z-faces, T at
 * cell centres; wall-normal velocities are zero and not stored.  T is the
 * centred temperature T - 1/2, so the x-walls hold +1/2 and -1/2.
 *
 * Inner product: volume weighted, <a,b> = sum V_q a_q b_q with V_q the
 * control volume of unknown q; P is orthogonal in it.
 *
 * Conventions for every call:
 *   - Vector arguments are DEVICE pointers owned by the caller (e.g. torch
 *     tensors), never freed or retained by the library, 256-byte alignment
 *     not required.  Host pointers are marked "host".
 *   - All work is enqueued on the HIP stream given to kv_create.  Calls that
 *     return host scalars synchronize that stream before returning.
 *   - Return value: KV_OK or an error code; nothing throws across the ABI.
 *     kv_last_error(ctx) gives a message for the last failed call.
 *   - Calls that need a base flow return KV_ESTATE before kv_set_base_flow.
 *   - The library allocates device memory only in kv_create (metrics,
 *     fast-diagonalization bases, two cell fields, reduction partials) and
 *     kv_set_preconditioner (the preconditioner's bases); kv_destroy frees
 *     it.  Every vector-sized scratch of a call (Krylov bases, solver
 *     vectors, the mixed form's scratch vector, the preconditioner's vectors)
 *     comes from a caller-owned workspace (kv_workspace_size,
 *     kv_set_workspace), so the caller's allocator (e.g. torch's) owns all
 *     memory that grows with the solver settings.
 *   - A context is not thread safe; calls on one context must not overlap.
 */
#ifndef KV_H
#define KV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kv_ctx kv_ctx;

enum kv_status {
  KV_OK = 0,
  KV_EINVAL = 1,      /* bad argument (sizes, grid, null pointer, flags) */
  KV_ENOMEM = 2,      /* device or host allocation failed */
  KV_EDEVICE = 3,     /* a HIP call failed (no gfx950 device, launch error) */
  KV_ENOCONV = 4,     /* iteration limit reached; outputs hold the last iterate */
  KV_ENONFINITE = 5,  /* NaN or Inf met in an input or an iterate */
  KV_ESTATE = 6       /* call needs kv_set_base_flow first */
};

/* Per-call flags.  KV_PROJECT: follow J by the projection P.  KV_MIXED
 * (kv_apply_jacobian, kv_project): the mixed-precision projection -- the
 * fast-diagonalization solve in FP32 storage on the FP32 matrix cores
 * (KV_MIXED_FD=bf16x3 in the environment: bf16x3 split products on the bf16
 * matrix cores), refined on the FP64 residual, the normalized divergence
 * max|net flux| / max|face flux| checked after every sweep from the second
 * until it is <= 1e-10 (KV_ENOCONV after 8 sweeps).  It needs every axis mirror-symmetric with an even cell count; on
 * other grids the FP64 projection is used.  The solvers take it through
 * kv_set_solver_projection. */
enum kv_flags { KV_PROJECT = 1u, KV_MIXED = 2u };

typedef struct {
  int nx, ny, nz;           /* cells per axis, each >= 2 */
  const double *xf, *yf, *zf; /* host: n+1 strictly increasing face
                               * coordinates per axis, first 0, last 1 */
  double Gr, Pr;            /* Gr >= 0, Pr > 0 */
} kv_params;

/* Create a context on the current HIP device: copies the grid, builds the
 * metrics and the fast-diagonalization bases (one symmetric eigenproblem
 * per axis, solved on the host).  hip_stream: a hipStream_t or NULL for the
 * default stream.  Errors: KV_EINVAL (bad grid), KV_EDEVICE, KV_ENOMEM. */
int kv_create(const kv_params* p, void* hip_stream, kv_ctx** out);
int kv_destroy(kv_ctx* ctx);

/* Packed size n and block offsets off[0..4] (u, v, w, T, end). host out. */
int kv_layout(const kv_ctx* ctx, int64_t* n, int64_t off[5]);

/* Caller-owned workspace.  The calls below carve their vector-sized scratch
 * from one device buffer that the caller allocates and keeps alive:
 *   KV_WS_PROJECT_MIXED         kv_apply_jacobian / kv_project with KV_MIXED
 *                               (1 packed vector)
 *   KV_WS_APPLY_PRECONDITIONER  kv_apply_preconditioner (1 vector)
 *   KV_WS_NEWTON                kv_newton_correction: 8 BiCGstab(2) vectors,
 *                               the GMRES(m) basis (m + 1, m of
 *                               kv_set_gmres_restart) and, with a
 *                               preconditioner set, 3 more vectors
 *   KV_WS_ARNOLDI               kv_arnoldi_leading_eigs: the Krylov basis
 *                               (krylov_dim + 1), 3 filter vectors, 2 (n_eigs
 *                               + 1) locked and Ritz vectors, the inner-solve
 *                               vectors of a spectral transform (below) and
 *                               the Hessenberg / Ritz-vector area
 * kv_workspace_size writes the bytes op needs (host out; krylov_dim and
 * n_eigs are read for KV_WS_ARNOLDI only; the Newton size depends on the
 * current GMRES restart and preconditioner, so query after setting them).
 * kv_set_workspace records dev_ptr (device, 8-byte aligned, bytes long;
 * NULL and 0 detach it); the library never frees it, and it must outlive
 * every call that uses it.  A call whose op needs more than is set returns
 * KV_EINVAL and does nothing.  One workspace serves every op (calls on a
 * context do not overlap).  Errors: KV_EINVAL (unknown op, bad sizes). */
enum kv_workspace_op {
  KV_WS_PROJECT_MIXED = 1,
  KV_WS_APPLY_PRECONDITIONER = 2,
  KV_WS_NEWTON = 3,
  KV_WS_ARNOLDI = 4,
  KV_WS_TIME_STEPS = 5        /* kv_time_steps: 4 vectors */
};
int kv_workspace_size(const kv_ctx* ctx, int op, int krylov_dim, int n_eigs, size_t* bytes);
int kv_set_workspace(kv_ctx* ctx, void* dev_ptr, size_t bytes);

/* Store the base flow X0 (device, packed, n values; copied).  Sec. 1: the
 * Jacobian is taken about the steady flow.  KV_ENONFINITE if X0 holds a NaN
 * or Inf. */
int kv_set_base_flow(kv_ctx* ctx, const double* X0);

/* F = P N(X0), the projected steady residual of Eqs. 1-6 at the base flow
 * (device out, n values).  norm (host, may be NULL) receives ||F||_W.  Used
 * by Newton's method (Sec. 1). */
int kv_residual(kv_ctx* ctx, double* F, double* norm);

/* y = J(X0) x, or y = P J(X0) x when flags has KV_PROJECT: one Krylov vector
 * of the paper's Newton and Arnoldi iterations (Sec. 3: divergence free and
 * satisfying all boundary conditions).  x, y: device, n values, must not
 * overlap.  With KV_PROJECT (FP64 form) the stencil also writes the scaled
 * net-flux divergence V^1/2 D y the projection starts from (Eq. 2 over each
 * cell). */
int kv_apply_jacobian(kv_ctx* ctx, const double* x, double* y, unsigned flags);

/* In place y <- P y (velocity block; T unchanged).  div_max (host, may be
 * NULL): normalized divergence max|net flux| / max|face flux| after the
 * projection.  sweeps (host, may be NULL): projection sweeps used (1 for
 * the FP64 projection, the refinement sweeps with KV_MIXED). */
int kv_project(kv_ctx* ctx, double* y, unsigned flags, double* div_max, int* sweeps);

/* kv_project with KV_MIXED for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same mixed projection of y in place, its scratch vector
 * in the library's static device array instead of a caller workspace.  The
 * array (64 MiB per GPU, held until the process ends) serves grids with
 * n <= 8,388,608 packed unknowns (128^3 and below); larger ones give
 * KV_EINVAL without touching y, as does a grid without the even/odd split
 * (it would take the FP64 projection, which needs no scratch: use
 * kv_project).  No allocation of any kind and no phase timing; div_max and
 * sweeps (host, may be NULL) as in kv_project.  All calls on one GPU share
 * the array, so calls that overlap on one GPU (other contexts, other
 * threads, other streams) race; each call writes every scratch entry it
 * reads. */
int kv_project_mixed_static(kv_ctx* ctx, double* y, double* div_max, int* sweeps);

/* <a, b>_W on the device, result to host *out. */
int kv_dot(kv_ctx* ctx, const double* a, const double* b, double* out);

/* y <- a x + b y on the device (packed vectors, n values; x may equal y).
 * a, b: host scalars. */
int kv_axpby(kv_ctx* ctx, double a, const double* x, double b, double* y);

/* Symmetry measures R_ref, R_2D, R_3D of Eqs. 7-9 (Sec. 2) of the packed
 * state X (device), over cell-centred theta = T - (1 - x).  host out[3]. */
int kv_symmetry_measures(kv_ctx* ctx, const double* X, double out[3]);

/* Symmetry classes of perturbations (Sec. 2, Eqs. 7-9; Sec. 4.1 tells the
 * two leading eigenmodes apart by them).  The cube is invariant under the reflection
 * y -> 1-y, (u,v,w,T) -> (u,-v,w,T), the 2-D rotation (x,z) -> (1-x,1-z),
 * (u,v,w,T) -> (-u,v,-w,-T), and their product, the 3-D centro-symmetry,
 * (u,v,w,T) -> -(u,v,w,T), each field read at the mirrored point (T centred).
 * A perturbation is EVEN under a map S if S x = x and ODD if S x = -x; its
 * centro-symmetry sign is the product of the other two.  At a base flow with
 * all three symmetries P J commutes with the maps and each eigenvector lies
 * in one class.  Give at most one bit per map; a map with no bit is free. */
enum kv_symmetry_class {
  KV_SYM_REF_EVEN = 1u << 4,  /* reflection kept */
  KV_SYM_REF_ODD = 1u << 5,   /* reflection broken (antisymmetric) */
  KV_SYM_ROT_EVEN = 1u << 6,  /* 2-D rotation kept */
  KV_SYM_ROT_ODD = 1u << 7    /* 2-D rotation broken (antisymmetric) */
};

/* y = Pi x, Pi the W-orthogonal projection onto the class given by sym: the
 * product over the restricted maps of (I + e S)/2, e = +1 (EVEN) or -1 (ODD).
 * x, y: device, packed, n values; y may equal x.  KV_EINVAL on bad bits or
 * when a restricted map mirrors an axis whose cell widths are not mirror-
 * symmetric (to 1e-12 of the largest width).  Needs no base flow.  Memory
 * bound: one read and one write of the vector. */
int kv_symmetry_project(kv_ctx* ctx, const double* x, double* y, unsigned sym);

typedef struct {
  int matvecs;      /* applications of P J */
  int cycles;       /* BiCGstab(2) cycles plus GMRES restarts */
  int used_gmres;   /* 1 if the GMRES continuation ran */
  double relres;    /* ||P J delta + F||_W / ||F||_W (recursive estimate;
                     * of the preconditioned system when a preconditioner is set) */
  int precond;      /* applications of the preconditioner M^-1 */
} kv_solve_info;

/* Newton correction (Sec. 1): delta with P J(X0) delta = -F, by BiCGstab(2)
 * (Sleijpen-Fokkema form, shadow vector = initial residual), continued by
 * restarted GMRES(m) (m = 40 unless kv_set_gmres_restart changed it) from
 * the current iterate after a breakdown or 50
 * cycles without a 10% residual reduction.  F is projected once more before
 * the solve, and a converged delta is projected once more at the end (the
 * Krylov combination is divergence-free only up to cancellation among its
 * terms).  Stops when relres <= tol or after max_matvec matvecs
 * (KV_ENOCONV, delta holds the last iterate).  delta0: optional initial
 * iterate (device, may be NULL, not aliasing delta).  F, delta: device, n
 * values.  info: host, may be NULL.  flags: 0, or KV_SYM_* bits (below):
 * the correction is sought in that symmetry class (right-hand side, every
 * Krylov vector and delta projected onto it; delta0 should lie in it).  A
 * steady state with the cube's symmetries (Sec. 2) has a correction in the
 * fully symmetric class (KV_SYM_REF_EVEN | KV_SYM_ROT_EVEN), and keeping
 * the solve there removes the eigenmodes of the other classes, one of which
 * turns singular where a symmetry-breaking real eigenvalue crosses zero.
 * (The mixed projection is chosen per context: kv_set_solver_projection.)
 * With a preconditioner set (kv_set_preconditioner) the solve is right
 * preconditioned: BiCGstab(2)/GMRES iterate on P J M^-1 and delta = delta0 +
 * M^-1 x. */
int kv_newton_correction(kv_ctx* ctx, const double* F, double tol, int max_matvec,
                         unsigned flags, const double* delta0, double* delta,
                         kv_solve_info* info);

/* Time integration of Eqs. 1-6 (Sec. 4.2 follows the oscillatory states that
 * the primary instability leads to by fully nonlinear computations; the
 * paper gives no scheme).  Semi-implicit steps: diffusion implicit, through
 * the Helmholtz solves of the Stokes/heat preconditioner (kv_set_
 * preconditioner's operators at shift s), advection and buoyancy explicit,
 * and every step projected by P, with F = P N(X) the steady residual:
 *   order 1:  X(t+dt) = X + M_{1/dt}^-1 F(X)
 *   order 2 (SBDF2, s = 3/(2 dt)):
 *     X(t+dt) = 2X - Xprev + M_s^-1 [ (2s/3)(Xprev - X) + 2F(X) - F(Xprev) ]
 * The steady states are exactly its fixed points.  X: device, packed, the
 * state at t (in) and at t + nsteps dt (out); Xprev: device, n values, the
 * state at t - dt (in, when start == 0) and at t + (nsteps - 1) dt (out).
 * start = 1 takes the first step at order 1 (Xprev is only written), then
 * order 2.  dt > 0 (host), nsteps >= 0.  The KV_WS_TIME_STEPS workspace
 * is used; the first call builds the preconditioner's bases if
 * kv_set_preconditioner has not; the preconditioner setting is kept.
 * KV_ENONFINITE if the state blows up (explicit advection: dt must respect
 * the convective CFL limit of the grid).  Needs no base flow. */
int kv_time_steps(kv_ctx* ctx, double dt, int nsteps, int start, double* X, double* Xprev);

/* Restart length m of the GMRES(m) that continues a stalled BiCGstab(2) in
 * kv_newton_correction (Sec. 1: BiCGstab(2) combined with GMRES); 10 <= m <=
 * 400, default 40.  A longer restart keeps the few eigenvalues of P J near
 * the imaginary axis, which a steady branch close to a Hopf point has, in the
 * Krylov space (restarting discards them); the KV_WS_NEWTON workspace grows
 * to m + 9 vectors.  Kept until changed. */
int kv_set_gmres_restart(kv_ctx* ctx, int m);

/* Deflated restarting of the GMRES(m) continuation (Morgan's GMRES-DR): k
 * harmonic Ritz vectors of the values of smallest modulus are kept from one
 * cycle to the next, with the residual, so that the few eigenvalues of the
 * (preconditioned) operator near zero -- which a steady branch near a Hopf
 * point has -- are not rebuilt every cycle.  0 <= k <= 62 (and at most m - 2),
 * default 0 (plain restarts).  The KV_WS_NEWTON workspace grows by one
 * vector and a Hessenberg area when k > 0.  Kept until changed. */
int kv_set_gmres_deflation(kv_ctx* ctx, int k);

/* Stagnation limit of the BiCGstab(2) part of kv_newton_correction (Sec. 1:
 * BiCGstab(2) combined with GMRES): after this many cycles without a 10%
 * drop of the residual norm below its best value the solve continues as
 * restarted GMRES(m) from the current iterate.  0 <= cycles <= 100000,
 * default 50; 0 hands the solve to GMRES before the first BiCGstab(2) cycle.
 * Kept until changed. */
int kv_set_bicgstab_stall(kv_ctx* ctx, int cycles);

/* Preconditioner of the Newton correction (an addition: the paper names no
 * preconditioner; Sec. 1 gives BiCGstab(2) with GMRES).  KV_PC_STOKES: right
 * preconditioning of P J by
 *   M^-1 r = ( P (sigma - nu Lap_v)^-1 r_vel , (sigma - kappa Lap_T)^-1 r_T ),
 * the discretization's own diffusion operators (no-slip velocity walls; T = 0
 * on the x-walls and adiabatic y- and z-walls), each inverted by fast
 * diagonalization (1-D eigenbases per axis, FP64 matrix cores): Stokes
 * preconditioning in Tuckerman's sense.  Kept until changed; KV_PC_NONE
 * switches it off.  sigma >= 0 (host).  The first KV_PC_STOKES call builds
 * the bases (9 symmetric eigenproblems on the host); the solve's three
 * extra vectors come from the KV_WS_NEWTON workspace. */
enum kv_preconditioner { KV_PC_NONE = 0, KV_PC_STOKES = 1 };
int kv_set_preconditioner(kv_ctx* ctx, int kind, double sigma);

/* y = M^-1 x with the preconditioner set on ctx (KV_ESTATE if none).
 * x, y: device, packed, n values; y may equal x. */
int kv_apply_preconditioner(kv_ctx* ctx, const double* x, double* y);

typedef struct {
  int krylov_dim;       /* m, Arnoldi steps per cycle, 2..400 */
  int n_eigs;           /* wanted leading eigenvalues, 1..m-1 */
  int max_matvec;       /* budget over all cycles and filters */
  int max_restarts;     /* 0: one Arnoldi cycle, Ritz values returned as is */
  int cheb_degree_max;  /* cap on the Chebyshev filter degree per restart */
  double tol;           /* converged when every wanted Ritz residual
                           <= tol * max |wanted Ritz value| */
  const double* v0;     /* device, n values: start vector (projected first) */
  unsigned flags;       /* 0, or KV_SYM_* bits: restrict the Krylov space
                           to that symmetry class (v0, every P J x and every
                           restart vector projected onto it); meaningful at
                           a base flow with all three symmetries */
  int keep;             /* 0: restart from one Chebyshev-filtered vector
                           (below).  n_eigs < keep <= krylov_dim - 2: restart
                           thick instead -- the real and imaginary parts of
                           the keep leading Ritz vectors (a pair whole, at
                           most 63 vectors), orthonormalized, start the next
                           cycle with the last Arnoldi vector after them, so
                           the cluster of weakly damped modes near the
                           imaginary axis stays in the Krylov space across
                           restarts (no filter, no locking) */
} kv_arnoldi_params;

typedef struct {
  int n_out;      /* values written: n_eigs, or n_eigs+1 to keep a pair whole */
  int matvecs;
  int restarts;
  int converged;  /* 1 if the tolerance was met */
  int relaxed_qr; /* cycles whose Hessenberg QR took a deflation only the
                     relaxed test allows (after 100 iterations without one
                     the test |h_{k,k-1}| <= eps (|h_kk| + |h_{k-1,k-1}|)
                     relaxes to sqrt(eps): a nearly defective Ritz cluster,
                     whose values are then fixed only to about sqrt(eps)
                     relative); 0 when every deflation met eps */
  int inner_matvecs; /* with a spectral transform: applications of P J by
                        its inner solves (matvecs then counts applications
                        of the transformed operator); 0 otherwise */
} kv_eig_info;

/* Leading eigenvalues (largest real part first, +Im before -Im within a
 * conjugate pair) of A = P J(X0) on divergence-free vectors, by restarted
 * Arnoldi (classical Gram-Schmidt twice, FP64) whose restart vector is
 * filtered by a Chebyshev polynomial on the ellipse around the unwanted Ritz
 * values (Sec. 1 and Sec. 3: Chebyshev-preconditioned Arnoldi, no shift-and-
 * invert).  The restart vector sums the real and imaginary parts of the
 * wanted Ritz vectors still open, each weighted by the inverse of its
 * predicted growth under the filter; converged values are locked in leading
 * order and their invariant subspaces deflated from later cycles and
 * filters.  The Hessenberg eigenproblem is solved on the GPU by Francis
 * double-shift QR.
 *   lam_re, lam_im, resid: host arrays of n_eigs+1 values; resid gets the
 *     Ritz residual norms (for a locked value, when it was locked).
 *   evecs: NULL, or device, (n_eigs+1) rows of n values: the eigenvector of
 *     output value q in row q, unit W-norm, sign not fixed; a conjugate pair
 *     q, q+1 as the real part (row q) and imaginary part (row q+1) of the
 *     eigenvector of the +Im member, turned so the two are W-orthogonal and
 *     the real part the longer.  Vectors of locked values are lifted from the
 *     deflated operator to A (a few extra P J x, counted in info->matvecs),
 *     and the workspace grows by n_eigs+1 vectors.
 *   info: host, may be NULL.
 * Not converged within max_matvec (or max_restarts > 0 restarts): KV_ENOCONV
 * with the last Ritz values (and their vectors).  A Hessenberg QR that does
 * not converge also gives KV_ENOCONV, with no values (info->n_out = 0;
 * matvecs and restarts count the work done). */
int kv_arnoldi_leading_eigs(kv_ctx* ctx, const kv_arnoldi_params* p, double* lam_re,
                            double* lam_im, double* resid, double* evecs, kv_eig_info* info);

/* Spectral transform of the thick-restarted Arnoldi (keep > 0) above, with
 * the Stokes/heat preconditioner of kv_set_preconditioner (an addition: the
 * paper runs Arnoldi on A itself, Sec. 3).  KV_ST_CAYLEY: Arnoldi runs on
 *   C = (A - pole)^-1 (A - zero),
 * which has the eigenvectors of A and maps an eigenvalue lambda to
 * theta = (lambda - zero) / (lambda - pole): values near the pole become
 * dominant and the stiff diffusive part of the spectrum (|lambda| >> |pole -
 * zero|) gathers near theta = 1.  Each application solves (A - pole) z = x by
 * restarted GMRES (the length of kv_set_gmres_restart, no deflated restarts),
 * right-preconditioned by M^-1 when a preconditioner is set, from z = 0 to
 * inner_tol relative residual within inner_max_matvec applications of P J
 * (else the Arnoldi call fails with KV_ENOCONV).  The wanted set is the
 * n_eigs values of largest |theta|; the convergence test applies tol to the
 * Ritz residuals of C relative to the largest wanted |theta|, and resid
 * reports those residuals.  Outputs are mapped back,
 * lambda = (pole theta - zero) / (theta - 1), and ordered as above (largest
 * real part first), with their eigenvectors.  pole: a real shift just right
 * of the wanted eigenvalues; zero: left of them, |pole - zero| about the
 * spread of the wanted part of the spectrum.  Kept until changed; KV_ST_NONE
 * switches it off.  The KV_WS_ARNOLDI workspace grows by gmres_m + 2 vectors
 * (+ 2 with a preconditioner): query kv_workspace_size after setting both.
 * Errors: KV_EINVAL (unknown kind, pole == zero, non-finite values,
 * inner_tol outside (0, 1), inner_max_matvec < 4); kv_arnoldi_leading_eigs
 * returns KV_EINVAL with a transform set and keep == 0. */
enum kv_spectral_transform { KV_ST_NONE = 0, KV_ST_CAYLEY = 1 };

/* Projection inside the solvers (kv_newton_correction, including its
 * preconditioner and final projection, and kv_arnoldi_leading_eigs,
 * including a spectral transform's inner solves): flags 0 for the FP64
 * projection (default) or KV_MIXED for the mixed form of kv_project
 * (normalized divergence <= 1e-10 after each projection).  The mixed form
 * is what the paper's mixed-precision configuration asks of the solvers;
 * it is an addition (the paper computes in FP64).  Kept until changed; the
 * KV_WS_NEWTON and KV_WS_ARNOLDI workspaces grow by one vector while
 * KV_MIXED is set.  KV_EINVAL for other flags, or KV_MIXED on a grid whose
 * axes are not mirror-symmetric of even size. */
int kv_set_solver_projection(kv_ctx* ctx, unsigned flags);
int kv_set_spectral_transform(kv_ctx* ctx, int kind, double pole, double zero, double inner_tol,
                              int inner_max_matvec);

/* Eigenvalues of a small upper Hessenberg matrix on the GPU: the Ritz
 * values of an Arnoldi cycle (Sec. 1) come from this Francis double-shift QR
 * (one wavefront; an exceptional shift pair every tenth iteration without a
 * deflation; after 100 iterations without a deflation the deflation test
 * relaxes from eps to sqrt(eps), which kv_eig_info.relaxed_qr counts in
 * Arnoldi).  H: host, m x m row-major, entries below the first subdiagonal
 * ignored; 1 <= m <= 400.  wr, wi: host, m values each, in the order the QR
 * deflates them (a complex pair as +Im, -Im in consecutive entries).
 * KV_ENONFINITE on a non-finite entry, KV_ENOCONV when the QR does not
 * converge (more than 30 max(10, m) iterations without a deflation, or 120
 * max(10, m) in all).  Needs no base flow. */
int kv_hessenberg_eigenvalues(kv_ctx* ctx, const double* H, int m, double* wr, double* wi);

/* Transfers for the learned Newton guess (kvnn.h).  Not part of the paper's
 * method: the paper starts each Newton solve from a converged state at a
 * nearby Gr (Sec. 1); these calls turn converged states into training targets
 * of a network and a network prediction back into a state.
 *
 * kv_cells_from_state: cell-centred fields of the packed state X (device) on
 * the grid coarsened by factor in every axis (nx, ny, nz multiples of factor;
 * factor 1 keeps the grid).  Per fine cell the centre values are
 * u = (u_west + u_east)/2 (walls 0), likewise v and w, and
 * theta = T - (1/2 - x_c) (the deviation from the conduction profile); a
 * coarse cell takes the volume-weighted mean over its factor^3 fine cells.
 * out (device FP32, 4 x (nz/f)(ny/f)(nx/f), [channel][z][y][x], channels
 * u, v, w, theta) = (mean - shift[c]) / scale[c].  shift, scale: host, 4
 * values, scale nonzero.  Non-finite X: KV_ENONFINITE. */
int kv_cells_from_state(kv_ctx* ctx, const double* X, int factor, const double shift[4],
                        const double scale[4], float* out);

/* kv_state_from_cells: the inverse direction.  cells (device FP32,
 * 4 x rz x ry x rx, as above) are values shift[c] + scale[c] * cells at the
 * network cell centres xc (rx), yc (ry), zc (rz) (host, strictly increasing
 * inside (0, 1)).  Every unknown of X (device, packed) becomes the trilinear
 * interpolant, in physical coordinates, at its own position (faces for u, v,
 * w; centres for T) over the node set extended by the walls 0 and 1 per
 * axis: velocities are 0 on every wall; theta is 0 on the x-walls and takes
 * the adjacent cell's value on the adiabatic y- and z-walls; T = theta +
 * 1/2 - x_c.  The result is not projected (kv_project does that). */
int kv_state_from_cells(kv_ctx* ctx, const float* cells, int rx, int ry, int rz, const double* xc,
                        const double* yc, const double* zc, const double shift[4],
                        const double scale[4], double* X);

/* kv_state_add_cell_increment: X += S(cells) - S(cells_ref), where S is the
 * interpolation of kv_state_from_cells (the shift and the conduction
 * profile cancel, so only scale is needed).  With cells and cells_ref the
 * network's predictions at Gr and at the Gr of a converged state X, this
 * moves X by the predicted change of the state between the two Gr.  X is
 * read and written (device, packed); cells and cells_ref are device FP32
 * arrays as in kv_state_from_cells.  The result is not projected. */
int kv_state_add_cell_increment(kv_ctx* ctx, const float* cells, const float* cells_ref, int rx, int ry,
                                int rz, const double* xc, const double* yc, const double* zc,
                                const double scale[4], double* X);

/* Device time per phase of the projected Jacobian, measured with HIP events
 * on the context's stream around each phase of every kv_apply_jacobian and
 * kv_project call while enabled.  enable = 1 starts the accounting (clearing
 * it), enable = 0 stops it; either way the sums since the last start are
 * returned (after synchronizing the stream) in ms[0..4) (host, may be NULL):
 * stencil, divergence, fast-diagonalization transforms (6 GEMM passes per
 * projection), gradient correction; calls[0..2) (host, may be NULL): number of
 * stencil applications and of projections measured.  For P J x the stencil
 * writes the divergence of its output itself (unless the environment sets
 * KV_FUSED_DIV=0), so "stencil" includes it and "divergence" is the pass
 * that completes the cells on the stencil's tile edges. */
int kv_timing(kv_ctx* ctx, int enable, double ms[4], int calls[2]);

/* Message of the last failed call on ctx (static text if ctx is NULL). */
const char* kv_last_error(const kv_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* KV_H */
