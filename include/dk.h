/*
 * dk.h - C ABI of libdk, the MI355X density-kernel library.
 *
 * libdk computes, on one GPU, the per-iteration hot path of the real-space
 * density-kernel method of Xu, Jing, Zhang, Pask & Suryanarayana (arXiv
 * 2112.08639, "SQ3"):
 *
 *   Chebyshev filter of a block of N_s grid vectors      (Sec. 4, 1st paragraph)
 *   orthonormalisation of the block                       (Sec. 4, 1st paragraph)
 *   subspace Hamiltonian H_s = <phi_i|H|phi_j>            (Sec. 3, before Eq. DsHsRelation)
 *   density kernel D_s = g(H_s) by Chebyshev expansion    (Eqs. ChebyshevExpansion,
 *     with the Fermi level from the electron count          ChebyshevCoeff, DMCFinal,
 *                                                           ThreeTermRecurrenceRelation,
 *                                                           FermiLevelCalc)
 *   band and entropy energies from the same expansion     (Sec. 4, E_band / E_ent expansions)
 *   density rho = 2 sum_i phi~_i phi_i                     (Eqs. phi_tilde, density:NewForm)
 *   Hellmann-Feynman forces                               (Eqs. force_nl:NewForm, force:NewForm)
 *
 * Discretisation.  A periodic orthorhombic cell lx x ly x lz holds an
 * nx x ny x nz grid, h_a = l_a / n_a, point (i,j,k) has flat index
 * i + nx*(j + ny*k).  H = -1/2 Lap_h + V_eff + sum_p gamma_p |chi_p><chi_p|
 * with the twelfth-order central-difference Laplacian (Sec. 5) and the
 * Kleinman-Bylander projectors of Eq. nonlocaloperator; the bra is the grid
 * quadrature h^3 sum_x.  Orbital blocks are normalised as h^3 X^T X = I,
 * so rho integrates (h^3 sum_x rho) to N_e.
 *
 * Memory.  Every large array is a caller-owned DEVICE pointer (libdk never
 * frees it).  A block of N_s grid vectors is column-major N_grid x N_s with
 * leading dimension ld >= N_grid: column c starts at X + c*ld.  Its element
 * type is double for a DK_PREC_FP64 context and float for a DK_PREC_MIXED
 * context.  N_s x N_s matrices (H_s, D_s) are column-major double with leading
 * dimension N_s.  The context owns only its copies of V_eff and the projector
 * tables.  Scratch memory is the caller's: query dk_workspace_bytes, allocate,
 * and hand it over with dk_set_workspace before the first compute call.
 *
 * Execution.  All work is issued on the stream given to dk_create, in stream
 * order.  A compute call returns after its work has finished (it synchronises
 * the stream), so device-detected failures are reported by the call that
 * caused them.  Contexts are independent; one context must not be used from
 * two threads at once.
 *
 * Errors.  Every function returns a dk_status and never aborts or throws.
 * Argument errors are detected on the host before any device work.  On error
 * dk_last_error(ctx) returns a message owned by the context, valid until the
 * next call on it.
 */
#ifndef DK_H
#define DK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dk_ctx dk_ctx;

typedef enum {
  DK_OK = 0,
  DK_ERR_ARG = 1,          /* invalid argument, detected on the host            */
  DK_ERR_DEVICE = 2,       /* no usable GPU, or a HIP runtime call failed        */
  DK_ERR_ALLOC = 3,        /* device allocation failed or workspace too small    */
  DK_ERR_NOT_SPD = 4,      /* Gram matrix not positive definite (rank-deficient) */
  DK_ERR_FERMI = 5,        /* electron count not bracketed: no Fermi level       */
  DK_ERR_NONFINITE = 6,    /* NaN or Inf met in an input or intermediate         */
  DK_ERR_STATE = 7,        /* call out of order (no potential / workspace yet)   */
  DK_ERR_CONVERGENCE = 8   /* spectral-bound iteration did not converge, or the
                              degree tail rule found no degree up to
                              DK_TAIL_MAX_DEGREE                                 */
} dk_status;

typedef enum { DK_PREC_FP64 = 0, DK_PREC_MIXED = 1 } dk_precision;

/* n_pl = 0 asks dk_density_kernel for the degree by the tail rule: the first of
 * 32, 64, 128, 256 whose Fermi-Dirac coefficient tail sum_{n < j <= 4n}
 * |c_j(mu)| is at most 1e-12 at that degree's Fermi level (the paper picks the
 * degree per system for accuracy, Sec. 5).  Buffers sized by degree (workspace,
 * tau) then hold DK_TAIL_MAX_DEGREE + 1 terms. */
#define DK_TAIL_MAX_DEGREE 256

/* Results of dk_density_kernel.  Spectrum and interval are those of H_s. */
typedef struct {
  double mu;          /* Fermi level (Ha)                                          */
  double lam_min;     /* smallest eigenvalue of H_s                                */
  double lam_max;     /* largest eigenvalue of H_s                                 */
  double chi;         /* (lam_max + lam_min)/2                                     */
  double xi;          /* (lam_max - lam_min)/2 (1 if H_s is a multiple of I)      */
  double e_band;      /* 2 sum'_j d_j tau_j                                        */
  double e_ent;       /* 2 sigma sum'_j e_j tau_j                                  */
  double n_count;     /* 2 sum'_j c_j tau_j at mu (equals N_e to bracket accuracy) */
  int n_pl;           /* degree of the expansion                                   */
  int bisect_iters;   /* mu search steps: 17-way bracketing, then Newton          */
  int bound_steps;    /* squaring steps taken for the spectral bounds              */
  int reserved;
} dk_fermi_info;

/* ---------------------------------------------------------------- setup -- */

/* Library version (major*10000 + minor*100 + patch). */
int dk_version(void);

/* Short name of a status code ("DK_OK", ...). Never NULL. */
const char* dk_status_name(int status);

/* Create a context on GPU `device` (HIP ordinal) for an nx x ny x nz periodic
 * grid over an lx x ly x lz cell (bohr).  precision selects the FP64 path or
 * the mixed path (FP32 blocks, FP32 stencil and projectors, split-BF16 MFMA for
 * the projection (two pieces, three products) and Phi*D (three pieces, six
 * products) products, FP64 Gram, Cholesky, bounds, expansion and Fermi
 * level).  stream is a hipStream_t (NULL = the default stream).
 * Requires 7 <= n_a (the stencil radius is 6), nx <= 1024, l_a > 0.
 * *ctx is set to NULL on failure.  DK_ERR_DEVICE if no GPU is present. */
dk_status dk_create(dk_ctx** ctx, int nx, int ny, int nz, double lx, double ly,
                    double lz, int precision, int device, void* stream);

/* Release a context and everything it allocated. NULL is accepted. */
dk_status dk_destroy(dk_ctx* ctx);

/* Message describing the last failure on ctx ("" if none). Owned by ctx. */
const char* dk_last_error(const dk_ctx* ctx);

/* Set V_eff (Ha, N_grid doubles, device pointer; copied).  Eq. KSeqn: the
 * local part V_xc + phi of the Hamiltonian on the grid.
 * DK_ERR_NONFINITE if it holds a NaN or Inf. */
dk_status dk_set_potential(dk_ctx* ctx, const double* veff_dev);

/* Set the Kleinman-Bylander projectors (Eq. nonlocaloperator), HOST arrays,
 * copied: projector p has values values[offsets[p] .. offsets[p+1]) at grid
 * indices indices[...] (0 <= index < N_grid, unique within a projector; the
 * periodic image sum is already applied), energy gamma[p] (Ha) and owning atom
 * atom[p] in [0, n_atoms).  n_proj = 0 removes the nonlocal term.
 * values are chi~_p at the grid points (bohr^-3/2). */
dk_status dk_set_projectors(dk_ctx* ctx, int n_proj, int n_atoms,
                            const int64_t* offsets, const int32_t* indices,
                            const double* values, const double* gamma,
                            const int32_t* atom);

/* Most projector channels per atom that dk_set_projector_model takes. */
#define DK_PROJ_MAX_CHANNELS 4

/* Build the Kleinman-Bylander projector tables (Eq. nonlocaloperator) on the
 * device from atom positions, in place of dk_set_projectors, so that moving
 * the atoms (an ionic step) needs no host-built tables.  Every atom carries
 * the same n_channels channels: channel k is the Gaussian
 * A_l exp(-r^2 / rc[k]^2) for l[k] = 0 (one projector) or that Gaussian times
 * the x, y, z components of r for l[k] = 1 (three projectors), with
 * A_0 = (2 / (pi rc^2))^(3/4) and A_1 = 2 A_0 / rc (unit norm in the
 * continuum), energy gamma[k] (Ha), truncated where r exceeds
 * rc sqrt(ln(1 / cutoff_rel)) and summed over periodic images.  Projector
 * order: atom-major, channels in the given order, l = 1 as x, y, z; the
 * result is the table dk_set_projectors takes for those values, up to the
 * rounding of the image sum and of exp.  pos: HOST, n_atoms x 3 (bohr, any
 * real coordinates; images are folded in), copied; l, rc, gamma: HOST,
 * n_channels entries.  Needs 1 <= n_channels <= DK_PROJ_MAX_CHANNELS,
 * l in {0, 1}, rc > 0, 0 < cutoff_rel < 1; n_atoms = 0 removes the nonlocal
 * term.  Tables of the previous call are reused when the projector count is
 * unchanged.  DK_ERR_NONFINITE for a NaN or Inf position or gamma. */
dk_status dk_set_projector_model(dk_ctx* ctx, int n_atoms, const double* pos,
                                 int n_channels, const int32_t* l,
                                 const double* rc, const double* gamma,
                                 double cutoff_rel);

/* Upper bound b >= lambda_max(H) in closed form: the kinetic symbol at the
 * zone corner, max V_eff, and sum over gamma_p > 0 of gamma_p h^3 |chi_p|^2.
 * Needs the potential (and projectors, if any). */
dk_status dk_spectrum_upper_bound(dk_ctx* ctx, double* b);

/* Bytes of device workspace the compute calls need for blocks of n_s columns
 * with leading dimension ld, and a density-kernel expansion of degree n_pl
 * (0: the tail rule, sized for DK_TAIL_MAX_DEGREE). */
dk_status dk_workspace_bytes(const dk_ctx* ctx, int n_s, int64_t ld, int n_pl,
                             size_t* bytes);

/* Hand over caller-owned device workspace (256-byte aligned, kept until the
 * next dk_set_workspace or dk_destroy).  Calls that need more return
 * DK_ERR_ALLOC. */
dk_status dk_set_workspace(dk_ctx* ctx, void* dev_ptr, size_t bytes);

/* ------------------------------------------------------------ hot path -- */

/* Y = H X for a block (one application of the discrete Hamiltonian, Eq.
 * KSeqn with Eq. nonlocaloperator).  X and Y must not overlap. */
dk_status dk_apply_h(dk_ctx* ctx, const void* X, void* Y, int64_t ld, int n_s);

/* In place X <- p_m(H) X: the degree-m Chebyshev filter (Sec. 4, first
 * paragraph) that damps [a, b] and is normalised to 1 at a0 < a, evaluated
 * with the scaled three-term recurrence
 *   Y_1 = (s_1/e)(H - c)X,  Y_{k+1} = (2 s_{k+1}/e)(H - c)Y_k - s_k s_{k+1} Y_{k-1},
 *   c = (a+b)/2, e = (b-a)/2, s_1 = e/(a0 - c), s_{k+1} = 1/(2/s_1 - s_k).
 * Mixed precision: the projector integrals of these applications take the
 * two-piece split-BF16 products (the result only spans the subspace that
 * dk_orthonormalize and dk_project then use); dk_apply_h and dk_project keep
 * the three-piece (FP32-level) ones.  Requires a0 < a < b, degree >= 1. */
dk_status dk_filter(dk_ctx* ctx, void* X, int64_t ld, int n_s, int degree,
                    double a, double b, double a0);

/* In place X <- X R^{-1} twice (CholQR2): G = h^3 X^T X = R^T R with R upper
 * triangular with positive diagonal.  Afterwards h^3 X^T X = I and X spans the
 * original columns.  DK_ERR_NOT_SPD if a Cholesky pivot is not positive
 * (X rank-deficient to working precision). */
dk_status dk_orthonormalize(dk_ctx* ctx, void* X, int64_t ld, int n_s);

/* hs (device, n_s x n_s FP64) <- h^3 X^T (H X), symmetrised as (H_s + H_s^T)/2.
 * The subspace Hamiltonian of Sec. 3 for an orthonormal block X. */
dk_status dk_project(dk_ctx* ctx, const void* X, int64_t ld, int n_s, double* hs_dev);

/* Smallest and largest eigenvalues of the symmetric hs (device, n_s x n_s), in
 * FP64 on the GPU, by shifted repeated squaring: with M = H_s - s I (s a
 * Gershgorin lower bound) and X_{k+1} = X_k^2 / tr(X_k^2), the quotient
 * <M, X_k^2>_F / tr(X_k^2) converges to lambda_max - s doubly exponentially;
 * lambda_min the same way from s' I - H_s with s' the Gershgorin upper bound; the
 * two sequences run side by side (one batched product per step), each until its
 * estimate is stationary to 1e-15 relative (DK_ERR_CONVERGENCE after 48 steps).
 * Used for the filter interval and for chi, xi of Eq. ChebyshevExpansion.  iters
 * (may be NULL) receives the squarings taken by the two sequences together. */
dk_status dk_spectral_bounds(dk_ctx* ctx, const double* hs_dev, int n_s,
                             double* lam_min, double* lam_max, int* iters);

/* Density kernel of Sec. 4: spectral bounds of hs, Hhat = (H_s - chi I)/xi,
 * T_0 = I, T_1 = Hhat, T_{j+1} = 2 Hhat T_j - T_{j-1} for j < n_pl,
 * tau_j = tr T_j, mu by bracketing (16 trial points per step, to a bracket of
 * 1e-14 max(1, |mu|)) on 2 sum'_j c_j(mu) tau_j = n_e with c_j the
 * K-node Gauss-Chebyshev values of Eq. ChebyshevCoeff (K = max(1024,
 * 4(n_pl+1))), then ds <- sum'_j c_j T_j and the band / entropy energies.
 * hs, ds: device n_s x n_s FP64 (may not overlap); tau_dev: device
 * n_pl+1 doubles (DK_TAIL_MAX_DEGREE+1 when n_pl = 0) or NULL; info: host,
 * info->n_pl is the degree used.  Requires 0 < n_e < 2 n_s, sigma > 0,
 * n_pl >= 0 (0: tail rule).  DK_ERR_FERMI if the electron count is not
 * bracketed; DK_ERR_CONVERGENCE if the tail rule finds no degree. */
dk_status dk_density_kernel(dk_ctx* ctx, const double* hs_dev, int n_s, double n_e,
                            double sigma, int n_pl, double* ds_dev, double* tau_dev,
                            dk_fermi_info* info);

/* rho (device, N_grid FP64) <- 2 sum_i (X D)_{x i} X_{x i}: Eqs. phi_tilde and
 * density:NewForm.  ds: device n_s x n_s FP64. */
dk_status dk_density(dk_ctx* ctx, const void* X, int64_t ld, int n_s,
                     const double* ds_dev, double* rho_dev);

/* dk_density for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result as dk_density, with the per-tile row partials in a
 * static device array of the library (128 MiB per GPU, held from the first
 * dk_create on that GPU until the process ends) instead of the context
 * workspace; no workspace needs to be set, and the call allocates nothing.
 * It holds ceil(n_s / 64) * N_grid * 8 bytes of partials in an FP64 context, and
 * ceil(n_s / 128) * N_grid * 8 bytes plus the three bf16 pieces of D (6 n_s
 * bytes per column, rows rounded up to 8 entries) in a mixed one; larger
 * problems get DK_ERR_ARG (use dk_density).  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (several streams or threads) race and give
 * wrong results; calls that follow each other in stream order are safe.  No
 * per-kernel timing (dk_profile_enable) is recorded for this call. */
dk_status dk_density_noalloc(dk_ctx* ctx, const void* X, int64_t ld, int n_s,
                             const double* ds_dev, double* rho_dev);

/* Band and entropy energies from the traces of the Chebyshev matrices (Sec. 4
 * expansions of E_band and E_ent; the entropy term carries the factor sigma of
 * Eq. FreeEnergy:NewForm): e_band = 2 sum'_j d_j tau_j,
 * e_ent = 2 sigma sum'_j e_j tau_j at Fermi level mu on the interval
 * [chi - xi, chi + xi].  tau_dev: device n_pl+1 doubles.  Outputs on host. */
dk_status dk_energy(dk_ctx* ctx, const double* tau_dev, int n_pl, double mu,
                    double chi, double xi, double sigma, double* e_band,
                    double* e_ent);

/* Hellmann-Feynman forces (host, 3*n_atoms doubles, atom-major x,y,z):
 *   nonlocal (Eq. force_nl:NewForm)
 *     f_I -= 4 sum_i sum_{p in I} gamma_p (h^3 chi_p^T x_i)(h^3 chi_p^T grad_h (X D)_i),
 *     grad_h the twelfth-order central first difference;
 *   local, if gradv_dev != NULL: f_I += h^3 sum_x rho(x) grad v_I(x) with
 *     gradv_dev device (n_atoms, 3, N_grid) FP64 (the gradient of each atom's
 *     local potential field) and rho_dev device N_grid FP64.
 * n_atoms must equal the projector tables' n_atoms when projectors are set. */
dk_status dk_forces(dk_ctx* ctx, const void* X, int64_t ld, int n_s,
                    const double* ds_dev, const double* rho_dev,
                    const double* gradv_dev, int n_atoms, double* forces);

/* Orbital terms of the Hellmann-Feynman stress tensor (host, 9 doubles each,
 * row-major [a][b], Ha/bohr^3), Eqs. stressIRe and stressIIIRe divided by the
 * cell volume |Omega| as in Eq. Stress:NewForm:
 *   kinetic[a][b]  = -2 sum_i h^3 sum_x (d_a x_i)(d_b (X D)_i) / |Omega|
 *   nonlocal[a][b] = ( -2 delta_ab sum_p gamma_p sum_i <chi_p,(X D)_i><chi_p,x_i>
 *                      -4 sum_p gamma_p sum_i <m^b_p, d_a (X D)_i><chi_p,x_i> ) / |Omega|
 * with d_a the twelfth-order central first difference along axis a,
 * <f,g> = h^3 sum_x f g, and m^b_p the first moment of projector p: the sum
 * over periodic images of chi_p(x - R - L) (x - R - L)_b.  ds: device
 * n_s x n_s FP64 (symmetric).  The nonlocal term needs tables built by
 * dk_set_projector_model (DK_ERR_STATE after dk_set_projectors with a nonzero
 * projector count); without projectors it is zero.  The other terms of the
 * stress (exchange-correlation and electrostatics) are not included. */
dk_status dk_stress(dk_ctx* ctx, const void* X, int64_t ld, int n_s,
                    const double* ds_dev, double* kinetic, double* nonlocal);

/* ------------------------------------------------------ self-consistency -- */
/* Support of the self-consistent loop around the steps above (Sec. 5 runs the
 * density-kernel evaluation inside SCF iterations).  All FP64, whatever the
 * context precision.  Electrostatics in the pseudocharge form of the paper's
 * real-space formulation (Sec. 2): the long-range local pseudopotential and
 * the Hartree potential are one potential V_c with
 *   -Lap_h V_c = 4 pi (rho + b),   b = sum_I b_I,
 *   b_I(x) = -z (pi rc^2)^(-3/2) sum_L exp(-|x - R_I - L|^2 / rc^2)
 * (the Gaussian charge whose potential is -z erf(r/rc)/r), Lap_h the same
 * twelfth-order periodic FD Laplacian as the kinetic operator.  Each atom also
 * contributes a short-range core term v_core(r) = -core_amp exp(-r^2/core_w2),
 * summed over periodic images. */
typedef struct {
  double z;         /* valence charge per atom                               */
  double rc;        /* pseudocharge width (bohr)                             */
  double core_amp;  /* core-term depth (Ha)                                  */
  double core_w2;   /* core-term width squared (bohr^2)                      */
} dk_local_model;

/* Energy integrals of one effective-potential update (h^3-weighted sums). */
typedef struct {
  double e_xc;          /* int rho eps_xc                                    */
  double int_rho_vc;    /* int rho V_c                                       */
  double int_rho_vxc;   /* int rho v_xc                                      */
  double e_es;          /* 1/2 int (rho + b) V_c - sum_I z^2/(sqrt(2 pi) rc) */
  double poisson_relres;/* final ||r|| / ||4 pi (rho + b - mean)||           */
  int poisson_iters;    /* CG iterations taken                               */
  int reserved;
} dk_scf_terms;

/* Set the atoms (pos: host, 3*n_atoms doubles, bohr, atom-major) and the local
 * model; builds b and v_core on the grid (owned by the context, N_grid FP64
 * each).  Replaces any previous atoms. */
dk_status dk_set_atoms(dk_ctx* ctx, int n_atoms, const double* pos,
                       const dk_local_model* model);

/* Copy b and/or v_core of the current atoms to caller device arrays (N_grid
 * FP64; either pointer may be NULL). */
dk_status dk_get_local_fields(dk_ctx* ctx, double* b_dev, double* vcore_dev);

/* Start density: the superposition of the atoms' Gaussian electron clouds,
 * rho_0 = -b (integral z n_atoms).  rho_dev: device N_grid FP64. */
dk_status dk_start_density(dk_ctx* ctx, double* rho_dev);

/* Linear solver of dk_poisson, dk_scf_potential and the Kerker solve of
 * dk_kerker_pulay_mix: conjugate gradients (the default), or alternating
 * Anderson-Richardson (Sec. 5 uses AAR for both solves): with the
 * Jacobi-scaled residual f_k = (b - A x_k) / diag A,
 *   x_{k+1} = x_k + omega f_k                          if (k+1) mod period != 0,
 *   x_{k+1} = x_k + beta f_k - (dX + beta dF) gamma_k  otherwise,
 * gamma_k minimising |f_k - dF gamma| over the differences of the last
 * `history` iterates (1 <= history <= 8).  The parameters are ignored for CG. */
#define DK_SOLVER_CG 0
#define DK_SOLVER_AAR 1
dk_status dk_set_linear_solver(dk_ctx* ctx, int solver, double omega, double beta, int history,
                               int period);

/* Solve -Lap_h v = 4 pi (src - mean(src)) by the context's linear solver from the
 * start vector in v_dev (device N_grid FP64, overwritten by the zero-mean
 * solution), until ||r|| <= tol ||4 pi (src - mean)||.  iters / relres (host,
 * may be NULL) receive the iterations and the final relative residual.
 * DK_ERR_CONVERGENCE after max_iter iterations. */
dk_status dk_poisson(dk_ctx* ctx, const double* src_dev, double* v_dev, double tol,
                     int max_iter, int* iters, double* relres);

/* LDA exchange-correlation of the unpolarised gas, Perdew-Wang 1992
 * correlation (Phys. Rev. B 45, 13244) and Slater exchange:
 * vxc_dev <- v_xc(rho) = d(rho eps_xc)/d rho; e_xc (host) <- h^3 sum rho eps_xc.
 * Densities <= 1e-20 contribute nothing. */
dk_status dk_xc(dk_ctx* ctx, const double* rho_dev, double* vxc_dev, double* e_xc);

/* Effective potential of an input density (needs dk_set_atoms):
 *   V_c  by dk_poisson with source rho + b, starting from vc_dev (in/out),
 *   veff = V_c + v_core + v_xc(rho)  -> veff_dev and the context potential
 *   (as dk_set_potential); energy integrals -> terms (host). */
dk_status dk_scf_potential(dk_ctx* ctx, const double* rho_dev, double* vc_dev,
                           double* veff_dev, double tol, int max_iter,
                           dk_scf_terms* terms);

/* Free energy of one SCF iteration in the Harris-Foulkes form with the input
 * density rho_in that produced V_eff (Eq. FreeEnergy:NewForm with the
 * pseudocharge electrostatics of Sec. 2):
 *   F = e_band + e_ent - int rho_in V_c - int rho_in v_xc + E_xc[rho_in] + e_es
 * from the energy integrals of dk_scf_potential (terms, host) and the band and
 * entropy energies of the density kernel.  xc_stress (host, 9 doubles, may be
 * NULL) <- the exchange-correlation term of the stress,
 * delta_ab (E_xc - int v_xc rho_in) / |Omega| (Eq. Stress:NewForm).
 * Host arithmetic only. */
dk_status dk_free_energy(dk_ctx* ctx, const dk_scf_terms* terms, double e_band, double e_ent,
                         double* free_energy, double* xc_stress);

/* Bytes of the caller-owned device state of dk_pulay_mix for `history`
 * stored pairs (1 <= history <= 8). */
dk_status dk_pulay_bytes(const dk_ctx* ctx, int history, size_t* bytes);

/* Pulay mixing of densities (device N_grid FP64 each; next may not alias in,
 * out).  With residuals F = out - in and the stored difference pairs
 * dR = in - in_prev, dF = F - F_prev of the last min(iter, history) calls:
 *   gamma = solution of (dF^T dF + 1e-12 tr/m I) gamma = dF^T F,
 *   next  = in + beta F - (dR + beta dF) gamma.
 * iter counts the calls on this state (0: start, no history).  residual
 * (host) <- ||F||_2 / ||out||_2.  Calls on one state must be in order. */
dk_status dk_pulay_mix(dk_ctx* ctx, void* state_dev, size_t state_bytes, int history,
                       int iter, double beta, const double* in_dev, const double* out_dev,
                       double* next_dev, double* residual);

/* Bytes of the caller-owned device state of dk_kerker_pulay_mix. */
dk_status dk_kerker_pulay_bytes(const dk_ctx* ctx, int history, size_t* bytes);

/* Kerker-preconditioned periodic Pulay mixing (the paper's SCF acceleration,
 * Sec. 5): the difference pairs are stored on every call as in dk_pulay_mix;
 * on every period-th call (iter + 1 divisible by period) gamma solves the
 * same normal equations, on the others gamma = 0, and
 *   next = (in - dR gamma) + beta P (F - dF gamma),
 *   P = (-Lap_h + k0^2)^{-1} (-Lap_h)   (k0 <= 0: P = I),
 * P applied by the context's linear solver (dk_set_linear_solver) from zero to
 * a relative residual tol (DK_ERR_CONVERGENCE after 20000 iterations).
 * restart != 0 selects the restarted form: the stored pairs are discarded after
 * every extrapolation, so each one uses the pairs gathered since the previous
 * one (period - 1 the first time, then period; needs period <= history).  P damps long wavelengths
 * and removes the mean.  residual (host) <- ||F||_2 / ||out||_2.  The state
 * must come from dk_kerker_pulay_bytes; calls on one state must be in order. */
dk_status dk_kerker_pulay_mix(dk_ctx* ctx, void* state_dev, size_t state_bytes, int history,
                              int iter, int period, int restart, double beta, double k0,
                              double tol, const double* in_dev, const double* out_dev,
                              double* next_dev, double* residual);

/* Electrostatic terms of the Hellmann-Feynman stress (Eq. Stress:NewForm) for
 * the pseudocharge model of dk_set_atoms (host, 9 doubles, row-major,
 * Ha/bohr^3):
 *   sigma_ab = ( (1/4 pi) <d_a V, d_b V> + sum_I <sum_L d_a b_I(x-R-L) (x-R-L)_b, V>
 *              + sum_I <rho, sum_L d_a v_core,I(x-R-L) (x-R-L)_b>
 *              + delta_ab (1/2) <b - rho, V> ) / |Omega|,
 * <f,g> = h^3 sum_x f g, d_a V the twelfth-order first difference, the
 * Gaussians b_I, v_core,I differentiated analytically (sums over periodic
 * images).  vc_dev: the zero-mean solution of -Lap_h V = 4 pi (rho + b) for
 * rho_dev (as dk_poisson or dk_scf_potential return it).  The continuum
 * self-energy does not depend on the strain and gives no term.  Needs
 * dk_set_atoms (DK_ERR_STATE otherwise). */
dk_status dk_electrostatic_stress(dk_ctx* ctx, const double* rho_dev, const double* vc_dev,
                                  double* sigma);

/* Local forces of the atoms set by dk_set_atoms (host, 3*n_atoms):
 *   f_I = h^3 sum_x grad b_I(x) vc(x) + h^3 sum_x rho(x) grad v_core,I(x),
 * the position derivative of 1/2 int (rho + b) V_c + int rho v_core. */
dk_status dk_local_forces(dk_ctx* ctx, const double* rho_dev, const double* vc_dev,
                          double* forces);

/* ------------------------------------------------- molecular dynamics -- */
/* Velocity-Verlet steps of Born-Oppenheimer dynamics (the paper's quantum
 * molecular dynamics, Sec. 5): v += (dt/2) f / M, R += dt v, new forces,
 * v += (dt/2) f / M.  Positions, velocities and forces are device arrays of
 * 3*n_atoms FP64 (atom-major x, y, z; bohr, bohr per a.u. of time, Ha/bohr). */

/* v_dev += half_dt * f_dev / mass */
dk_status dk_verlet_kick(dk_ctx* ctx, int n_atoms, double* v_dev, const double* f_dev,
                         double half_dt, double mass);

/* Isokinetic half kick (the Gaussian thermostat of the Sec. 5 transport runs):
 * v_dev (3 n_atoms, device) <- the exact flow over time tau of
 *   dv/dt = f/M - alpha v,  alpha = (f . v) / (M v . v)  (sums over all 3N components),
 * with the forces f_dev held fixed: with g = f/M, a = g.v/v.v, b = g.g/v.v,
 * w = sqrt(b) tau, v <- (v + g s)/s' where s = a (cosh w - 1)/b + sinh(w)/sqrt(b)
 * and s' = a sinh(w)/sqrt(b) + cosh w.  The kinetic energy is unchanged.  If
 * every velocity is zero, v is left as it is (the friction term is undefined). */
dk_status dk_isokinetic_kick(dk_ctx* ctx, int n_atoms, double* v_dev, const double* f_dev,
                             double tau, double mass);

/* x_dev += dt * v_dev (positions are not wrapped: every field is periodic) */
dk_status dk_verlet_drift(dk_ctx* ctx, int n_atoms, double* x_dev, const double* v_dev,
                          double dt);

/* e (host) <- (mass / 2) sum v^2 */
dk_status dk_kinetic_energy(dk_ctx* ctx, int n_atoms, const double* v_dev, double mass,
                            double* e);

/* ------------------------------------------------------------ transport -- */
/* Green-Kubo transport coefficients (Sec. 5, high-temperature QMD):
 *   D(t)   = (1/3N) sum_i int_0^t <v_i(tau) . v_i(0)> dtau,
 *   eta(t) = (|Omega| / k_B T) int_0^t (1/5) sum_m <s_m(tau) s_m(0)> dtau,
 * s_m the five independent deviatoric stress components.  The ensemble
 * average of one run is the average over time origins. */

/* corr_dev[k] (k < max_lag) <- sum_c sum_{t0 < T-k} s[(t0+k) n_comp + c] s[t0 n_comp + c]
 *                              / (n_comp (T - k))
 * for a series_dev of T = n_steps samples of n_comp components (device FP64,
 * step-major); integral_dev (may be NULL) <- scale times the trapezoid running
 * integral of corr on the spacing dt (integral[0] = 0).  The 3N velocity
 * components (scale 1) give C = VACF / 3 and D(t_k); the five deviatoric
 * components (scale |Omega| / k_B T) give the SACF and eta(t_k).
 * Needs 0 < max_lag <= n_steps, n_comp > 0 (and dt > 0 with an integral). */
dk_status dk_time_correlation(dk_ctx* ctx, const double* series_dev, int64_t n_steps, int n_comp,
                              int max_lag, double dt, double scale, double* corr_dev,
                              double* integral_dev);

/* s_dev (device, n_steps x 5) <- the deviatoric components s_12, s_23, s_31,
 * (s_11 - s_22)/2, (s_22 - s_33)/2 of the microscopic stress of each step:
 * sigma_dev (device, n_steps x 9, row-major 3 x 3; s_12 is entry [0][1],
 * s_23 [1][2], s_31 [2][0]) minus, if v_dev (device, n_steps x 3 n_atoms) is not NULL, the
 * ions' momentum flux sum_I mass v_Ia v_Ib / |Omega| (|Omega| the context cell). */
dk_status dk_deviatoric_stress(dk_ctx* ctx, const double* sigma_dev, const double* v_dev,
                               int n_atoms, double mass, int64_t n_steps, double* s_dev);

/* ------------------------------------------------------ learned start -- */
/* A per-grid-point network predicts the SCF start density from Gaussian
 * descriptors of the atomic environment.  Parameters are one FP32 vector
 * (device), per layer W (n_out x n_in, row-major) then b, for the layers
 * n_in -> hidden (x n_hidden_layers, SiLU) -> 1 (softplus).  Products run on
 * MFMA: DK_MLP_BF16 rounds weights and activations to BF16 with FP32
 * accumulation; DK_MLP_F32 uses FP32 MFMA (for verification).  Activations
 * and inputs are feature-fastest: u[k + p * n_in]. */
typedef struct {
  int n_in;             /* descriptor channels                               */
  int hidden;           /* width of the hidden layers (<= 64 per MFMA tile)  */
  int n_hidden_layers;  /* 1..8                                              */
} dk_mlp_shape;

#define DK_MLP_BF16 0
#define DK_MLP_F32 1

/* Number of parameters of the network. */
dk_status dk_mlp_param_count(const dk_mlp_shape* shape, int64_t* count);

/* Bytes of caller-owned device workspace for dk_mlp_loss_grad / dk_mlp_forward
 * over n_points points and for dk_mlp_density. */
dk_status dk_mlp_workspace_bytes(const dk_mlp_shape* shape, int64_t n_points, size_t* bytes);

/* Descriptors of the atoms at pos (host, 3*n_atoms, bohr):
 * desc[x * n_w + k] = sum_J sum_L exp(-|x - R_J - L|^2 / (2 w_k^2)) with
 * widths w (host, n_w); desc_dev: device N_grid x n_w FP32. */
dk_status dk_descriptors(dk_ctx* ctx, int n_atoms, const double* pos, int n_w,
                         const double* widths, float* desc_dev);

/* Per-channel mean and inverse standard deviation (device, n_w FP64 each; a
 * constant channel gets 1) of n_points descriptor rows (device, n_points x n_w
 * FP32), accumulated in FP64 (two passes). */
dk_status dk_descriptor_stats(dk_ctx* ctx, const float* desc_dev, int64_t n_points, int n_w,
                              double* mean_dev, double* inv_std_dev);

/* Training batch: for j < n_pts with q = idx[j] (device int64; NULL: q = j),
 * u[k + j n_w] = (desc[q n_w + k] - mean_k) inv_std_k and, if rho_dev is not
 * NULL, t[j] = scale * rho[q] (rho FP64).  desc / rho may stack several
 * snapshots. */
dk_status dk_mlp_gather(dk_ctx* ctx, const float* desc_dev, const double* rho_dev, int n_w,
                        const int64_t* idx_dev, int64_t n_pts, const double* mean_dev,
                        const double* inv_std_dev, double scale, float* u_dev, float* t_dev);

/* loss = mean_p (softplus(net(u_p)) - t_p)^2 (host) and, if grad_dev is not
 * NULL, its gradient with respect to the parameters (device FP32, layout of
 * the parameter vector) by backpropagation. */
dk_status dk_mlp_loss_grad(dk_ctx* ctx, const dk_mlp_shape* shape, int mode,
                           const float* params_dev, const float* u_dev, const float* t_dev,
                           int64_t n_pts, float* grad_dev, double* loss, void* ws,
                           size_t ws_bytes);

/* y_dev (device FP64, n_pts) <- softplus(net(u_p)). */
dk_status dk_mlp_forward(dk_ctx* ctx, const dk_mlp_shape* shape, int mode,
                         const float* params_dev, const float* u_dev, int64_t n_pts,
                         double* y_dev, void* ws, size_t ws_bytes);

/* One Adam step (Kingma & Ba) on n parameters (device FP32): step t >= 1,
 * bias-corrected moments, theta -= lr mhat / (sqrt(vhat) + eps). */
dk_status dk_adam_step(dk_ctx* ctx, int64_t n, float* params_dev, float* m_dev, float* v_dev,
                       const float* grad_dev, int t, double lr, double beta1, double beta2,
                       double eps);

/* Start density on the grid from one snapshot's descriptors:
 * rho = n_e y / (h^3 sum_x y), y = softplus(net((desc - mean) inv_std)). */
dk_status dk_mlp_density(dk_ctx* ctx, const dk_mlp_shape* shape, int mode,
                         const float* params_dev, const float* desc_dev, const double* mean_dev,
                         const double* inv_std_dev, double n_e, double* rho_dev, void* ws,
                         size_t ws_bytes);

/* Kernel kinds reported by dk_profile_read. */
typedef enum {
  DK_K_STENCIL = 0,      /* fused local stencil + Chebyshev update        */
  DK_K_NL_GATHER = 1,    /* projector integrals h^3 chi^T X (+ reduction)  */
  DK_K_NL_SCATTER = 2,   /* Y += chi (gamma C)                             */
  DK_K_GRAM = 3,         /* Gram product and reduction                     */
  DK_K_PROJECT = 4,      /* X^T (H X) product and reduction                */
  DK_K_CHOLESKY = 5,     /* blocked Cholesky and triangular inverse        */
  DK_K_ORTH_APPLY = 6,   /* X R^{-1}                                       */
  DK_K_BOUNDS = 7,       /* spectral bounds of H_s                         */
  DK_K_FOE_GEMM = 8,     /* Chebyshev recurrence products                  */
  DK_K_FERMI = 9,        /* traces, quadrature, bisection, D assembly      */
  DK_K_DENSITY = 10,     /* X D product with the row-sum epilogue          */
  DK_K_FORCES = 11,      /* force contractions                             */
  DK_K_OTHER = 12,
  DK_K_POISSON = 13,     /* CG iterations of the electrostatic solve       */
  DK_K_SCF_FIELDS = 14,  /* atom fields, LDA, effective potential, forces  */
  DK_K_MIX = 15,         /* Pulay mixing, and the learned-start network     */
  DK_K_STRESS = 16,      /* kinetic and nonlocal stress contractions       */
  DK_K_COUNT = 17
} dk_kernel_kind;

/* Turn per-kernel timing on (1) or off (0) and clear the counters.  When on,
 * every kernel launch of the context is bracketed by a pair of HIP events on
 * the context stream; times are accumulated per dk_kernel_kind. */
dk_status dk_profile_enable(dk_ctx* ctx, int on);

/* Accumulated GPU milliseconds and launch counts per kernel kind since the
 * last dk_profile_enable (ms and counts: DK_K_COUNT entries each, host). */
dk_status dk_profile_read(dk_ctx* ctx, double* ms, int64_t* counts);

/* Milliseconds of GPU time of the last call of each kind (filter, orthonormalize,
 * project, bounds, density_kernel, density, energy, forces), measured with
 * HIP events on the context stream.  n <= 8 values are written. */
dk_status dk_get_timings(const dk_ctx* ctx, double* ms, int n);

#ifdef __cplusplus
}
#endif

#endif /* DK_H */
