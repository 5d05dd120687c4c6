/*
 * mrcm.h -- C ABI of the MI355X (gfx950) implementation of the Multiscale
 * Robin Coupled Method (MRCM): batched construction of the Multiscale Basis
 * Functions (MBFs), assembly and solution of the interface coupling system,
 * and reconstruction of the pressure and velocity fields.
 *
 * Problem statement: single-phase Darcy flow, eqs. (2.3)-(2.6) of the paper
 * with a diagonal, anisotropic (mobility-scaled) permeability K-hat, on a
 * Cartesian grid discretised by two-point fluxes, eqs. (2.9)-(2.12).  The MRCM
 * is Algorithm 2 ("Pseudocode for the DD Multiscale mixed method"): local
 * Robin problems (2.13)/(2.14), weak continuity (2.15)/(2.16), interface
 * system (2.18)-(2.22), reconstruction (2.23), MBF systems (2.25)/(2.26).
 *
 * General conventions
 *  - Cells are indexed c = i + nx*(j + ny*k) (x fastest).  Faces of a cell are
 *    ordered -x, +x, -y, +y, -z, +z.
 *  - Pointers marked [dev] are device pointers (HIP global memory) that must
 *    stay valid until the work enqueued on `stream` has completed.  Pointers
 *    marked [host] are read or written before the call returns.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *  - All floating point arguments and results are IEEE double.
 *  - Errors: every entry point returns an mrcm_status.  Argument errors are
 *    detected on the host before anything is enqueued (MRCM_EINVAL, with a
 *    message in mrcm_last_error()).  Numerical failures are raised through a
 *    device status word that the call reads back at its end (one stream
 *    synchronisation).  No C++ exception crosses the ABI.
 *  - Handles are not thread-safe; distinct handles may be used concurrently on
 *    distinct streams.  Destroy functions synchronise the handle's last stream.
 */
#ifndef MRCM_H
#define MRCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MRCM_OK = 0,
  MRCM_EINVAL = -1,        /* invalid argument (message in mrcm_last_error) */
  MRCM_ENOMEM = -2,        /* device allocation failed */
  MRCM_ENOTSPD = -3,       /* non-positive pivot in a local factorisation */
  MRCM_ENOCONV = -4,       /* iterative refinement did not reach its tolerance */
  MRCM_ESINGULAR = -5,     /* zero pivot in the interface factorisation */
  MRCM_EHIP = -6,          /* HIP runtime error */
  MRCM_EUNSUPPORTED = -7   /* valid request outside this build's limits */
} mrcm_status;

/* Wall boundary types (eqs. (2.5), (2.6)). */
enum { MRCM_WALL_NOFLOW = 0, MRCM_WALL_DIRICHLET = 1, MRCM_WALL_NEUMANN = 2 };

/* Precision of the local factorisations. */
enum { MRCM_FP64 = 0,          /* FP64 band Cholesky and solves */
       MRCM_FP32_IR = 1,       /* FP32 factor and solves + FP64 refinement */
       MRCM_PCG = 2 };         /* per-column Jacobi-preconditioned CG (FP32
                                  inner iterations, FP64 residual), FP64 band
                                  Cholesky for the subdomains it leaves */

/* Robin parameter on Gamma (mrcm_options.beta_mode); eq. (3.1) leaves open
 * which K and H apply where the two sides of an interface differ. */
enum { MRCM_BETA_PER_SIDE = 0,  /* each side its own: alpha H_own / K_d(own cell) */
       MRCM_BETA_FACE = 1 };    /* one value per fine face, shared by both sides:
                                   alpha H~ / K~ with H~ the harmonic mean of the two
                                   subdomains' extents along the normal and K~ that of
                                   the two cells' K_d across the face */

/* What an MBF handle keeps after its build (mrcm_options.keep), deciding the
 * reconstruction of Loop 2: by the combination (2.23) of the kept MBFs, or by
 * solving the local problems again with the interface data, the second
 * option the paper gives after (2.23). */
enum { MRCM_KEEP_FACTORS = 1,   /* the local band factors */
       MRCM_KEEP_MBFS = 2 };    /* the MBFs X_l (reconstruction by combination) */

/* How the ragged launches of loop 1 take their subdomains (mrcm_options.launch_mode). */
enum { MRCM_LAUNCH_GRID = 0,    /* one workgroup per subdomain or work item */
       MRCM_LAUNCH_QUEUE = 1 }; /* persistent workgroups over a device work queue */

/*
 * The Darcy problem (Sec. 2.1).  All arrays have N = nx*ny*nz entries.
 *  kx, ky, kz  [dev] diagonal of K-hat per cell; must be positive and finite.
 *  q           [dev] total volumetric source rate per cell (f times cell volume).
 *  wall_type   per wall, -x..+z: MRCM_WALL_*.
 *  wall_value  [dev] per wall: NULL (all zero) or the wall's data, indexed by
 *              the two in-plane cell coordinates, lower axis fastest
 *              (-x/+x: j + ny*k; -y/+y: i + nx*k; -z/+z: i + nx*j).  Dirichlet:
 *              pressure g_p; Neumann: outward normal velocity g_u.
 *  pin_cell    cell whose pressure is fixed to 0 (gauge), or -1.  Required when
 *              no wall is Dirichlet.
 */
typedef struct {
  int32_t nx, ny, nz;
  double hx, hy, hz;
  const double *kx, *ky, *kz;
  const double *q;
  int32_t wall_type[6];
  const double *wall_value[6];
  int64_t pin_cell;
} mrcm_problem;

/*
 * Non-overlapping tensor-product partition (Sec. 2.2).  Subdomain
 * l = sx + ndx*(sy + ndy*sz) covers cut_x[sx] <= i < cut_x[sx+1], etc.
 *  cut_x/y/z [host] ndx+1 / ndy+1 / ndz+1 strictly increasing offsets from 0
 *            to nx / ny / nz.
 */
typedef struct {
  int32_t ndx, ndy, ndz;
  const int32_t *cut_x, *cut_y, *cut_z;
} mrcm_partition;

/*
 * Interface space V_H (Sec. 2.2.2, piecewise constants on patches obtained by
 * condensing fine faces).  For an interface normal to axis d with tangential
 * axes a < b, (na, nb) patches split it along a and b; n cells split into k
 * patches give the first (n mod k) patches ceil(n/k) cells and the rest
 * floor(n/k).  (0, 0) asks for one patch per fine face.
 *  uniform_split[d] = {na, nb} for every interface normal to axis d.
 *  split [host] optional override, one {na, nb} per interface, or NULL.
 *        Interfaces are listed x-normal, then y-normal, then z-normal, each in
 *        increasing order of the lower subdomain id.  Patches are numbered in
 *        the same order, pa + na*pb within an interface; the interface
 *        unknowns are X = (pi^p_0 .. pi^p_{NV-1}, pi^u_0 .. pi^u_{NV-1}).
 */
typedef struct {
  int32_t uniform_split[3][2];
  const int32_t *split;
} mrcm_iface_space;

/*
 * alpha        Robin parameter, eq. (3.1): beta_f = alpha * H_d / K_d(c) per side,
 *              H_d the own subdomain's extent along the face normal (physical
 *              length) and K_d(c) the own cell's permeability; alpha > 0.
 * precision    MRCM_FP64 or MRCM_FP32_IR.
 * ir_tol       FP32_IR: stop when every column's relative FP64 residual
 *              ||R - M X|| / ||R|| is at most ir_tol (<= 0 selects 1e-13), or
 *              is within the rounding bound of its own evaluation,
 *              ||R - M X|| <= 8u ||s|| with s_r = |R_r| + sum_j |M_rj X_j| and
 *              u = 2^-53 (no sweep can improve such a column further; on
 *              strongly heterogeneous or nearly Neumann local problems that
 *              floor can lie above 1e-13).
 * ir_max_iter  FP32_IR: refinement sweeps (<= 0: 30).  If they stop short of
 *              ir_tol, every column is polished once by the conjugate-gradient
 *              kernel of MRCM_PCG (FP64 residual, FP32 inner iterations, up to
 *              1000 of them, from the current X) when the blocks fit it
 *              (bandwidth <= 112, at most 2048 cells); MRCM_ENOCONV if a
 *              column is still above both ir_tol and its rounding floor.
 * fp64_refine  FP64: fixed number of FP64 refinement sweeps (residual
 *              R - A X from the coefficients, correction with the same factor)
 *              after the direct solves; 0 for none.
 * PCG (iterative local solves; the paper's "LocalSolver" paragraph of the
 * implementation section (`sec:code_overview`) compares a direct LDL^T with preconditioned
 * GMRES for the multi-right-hand-side local problems and keeps the direct one
 * at these sizes, table `tab:comp_local_mumps_hypre`):
 *              every right-hand-side column is solved by conjugate gradients on
 *              the Jacobi-scaled local matrix, with FP32 inner iterations
 *              restarted from the FP64 residual R - A X, until
 *              ||R - A X|| / ||R|| <= ir_tol (<= 0 selects 1e-10, which keeps
 *              the end-to-end pressure within 1e-6 of the direct solution on
 *              the 40x40x20 and 60x220x85 workloads; 1e-8 leaves ~1e-5).  A subdomain
 *              with any column not converged within pcg_max_iter inner
 *              iterations (<= 0: 50) is factorised by the FP64 band Cholesky
 *              and all its columns are solved directly instead, followed by
 *              fp64_refine refinement sweeps as in the FP64 form.
 * pcg_max_iter PCG: inner-iteration budget per column.
 * pcg_x0       PCG: [dev] starting guess in the layout of the MBFs (per
 *              subdomain l in id order, n_cells x n_rhs, row-major in the
 *              local row ordering, the same layout as mrcm_copy_mbfs), or NULL
 *              for zero.  A column whose guess (after pcg_x0_scale) leaves a
 *              residual larger than its right-hand side starts from zero
 *              instead.  Read during the call only.
 * solve_tiles  tiles of 16 right-hand-side columns per work item of the band
 *              solves (0: the largest, 3): fewer give more, smaller items.
 * solve_group  FP64 with refinement: subdomains whose first solve starts when
 *              the factorisation's whole rounds are done (rounded down to a
 *              multiple of 8); 0 derives it from the kernels' occupancy, -1
 *              turns the two-stream pipeline off.  Both are set by
 *              mrcm_autotune; a handle's geometry includes them.
 * pcg_x0_scale PCG: nonzero to replace each column's starting guess v by
 *              c v with c = (v, b) / (v, A v), the multiple of v closest to the
 *              solution in the A-norm (for a guess known only up to scale,
 *              such as the network output of mrcm_nn.h).
 * beta_mode    MRCM_BETA_PER_SIDE (0, the default) or MRCM_BETA_FACE.
 * keep         MRCM_KEEP_* bits; 0 selects MRCM_KEEP_FACTORS | MRCM_KEEP_MBFS.
 *              Without MRCM_KEEP_MBFS, mrcm_reconstruct solves every local
 *              problem again (particular data plus G(pi) on Gamma) with the
 *              kept factors and the form's refinement sweeps (FP64: fp64_refine;
 *              FP32: the build's, at least 3), and mrcm_copy_mbfs refuses.  The
 *              build forms every MBF either way (the flux blocks reduce them),
 *              so the handle's memory does not change.  The conjugate-gradient
 *              form keeps no factors and needs MRCM_KEEP_MBFS.
 * iface_panel  16-column blocks per panel of the multifrontal interface
 *              factorisation, 1 to 4 (0: 4): each panel's trailing update is
 *              one rank-(16 iface_panel) product.  Set by mrcm_autotune; an
 *              interface handle takes the value of its MBF handle.
 * launch_mode  MRCM_LAUNCH_GRID (0, the default): the ragged launches of the
 *              direct forms' factorisation and band solves run one workgroup
 *              per subdomain or work item; MRCM_LAUNCH_QUEUE (1): a
 *              persistent grid of resident workgroups takes the same items,
 *              in the same cost order, from a device work queue (one atomic
 *              counter per XCD); no workgroup waits on another.  The results
 *              are bitwise the same.  Set by mrcm_autotune.
 */
typedef struct {
  double alpha;
  int32_t precision;
  double ir_tol;
  int32_t ir_max_iter;
  int32_t fp64_refine;
  int32_t pcg_max_iter;
  const double *pcg_x0;
  int32_t pcg_x0_scale;
  int32_t solve_tiles;
  int32_t solve_group;
  int32_t beta_mode;
  uint32_t keep;
  int32_t iface_panel;
  int32_t launch_mode;
} mrcm_options;

typedef struct mrcm_mbfs mrcm_mbfs;           /* local factors, MBFs, Gamma-flux blocks */
typedef struct mrcm_interface mrcm_interface; /* interface band matrix and right-hand side */

typedef struct {
  int32_t n_sub;          /* subdomains */
  int32_t n_patch;        /* patches N_V; the interface system has 2*N_V unknowns */
  int64_t n_cells;        /* N */
  int64_t n_mbfs;         /* sum over subdomains of 2|I^l| (MBF solves, particular solves excluded) */
  int64_t n_rhs;          /* sum over subdomains of 2|I^l| + 1 */
  int32_t max_band;       /* largest local bandwidth b_l */
  int32_t max_rhs;        /* largest m_l */
  int32_t precision;
  int32_t ir_iters;       /* refinement sweeps of the last build (FP32_IR) */
  double ir_residual;     /* largest relative column residual after the last build
                             (above ir_tol only for columns at their rounding floor) */
  double factor_flops;    /* sum_l sum_k (b_k^2 + 2 b_k + 1), the band Cholesky count */
  double solve_flops;     /* sum_l 4 N_l b_l m_l (forward + backward band solves) */
  int64_t device_bytes;   /* device memory held by the handle */
  int32_t pcg_fallback;   /* PCG: subdomains solved by the band Cholesky in the last build */
  int64_t pcg_iters;      /* PCG: inner iterations of the last build, summed over columns */
} mrcm_info;

/* Per-subdomain layout, for tests and tools.  The local row ordering puts the
 * box's shortest axis fastest: r = t0 + n0*(t1 + n1*t2), t_k the cell
 * coordinate along axis ax[k] relative to lo[ax[k]], ties broken by lower axis
 * id; the lower bandwidth is b = n0*n1. */
typedef struct {
  int32_t lo[3], ext[3];
  int32_t ax[3];
  int32_t n_cells, band, n_rhs, n_patch;
  int32_t pin_local;      /* local row of the pinned cell, or -1 */
  int32_t solve_group;    /* FP64 (with refinement) and FP32 forms: 0 if the subdomain's first
                             solve is in the 'solve' stage's launch, 1 if it runs in the
                             'refine' stage (see below) */
} mrcm_subdomain_info;

/*
 * Loop 1 of Algorithm 2: for every subdomain, assemble the local matrix
 * A^H_l (TPFA inside, Robin terms on Gamma, wall terms), factorise it once
 * (band Cholesky), and solve the 2|I^l| + 1 systems (2.25)/(2.26); then
 * reduce the MBF fluxes over each patch into the blocks
 *   F[i,col]  = sum_{f in i} Q_f[col],   Fb[i,col] = sum_{f in i} beta_f Q_f[col]
 * with Q_f = T_f (p_c - G_f), T_f = A_d / (h_d/(2 K_d(c)) + beta_f).
 * Right-hand-side columns: 0 particular problem (G = 0); 1..n P-type MBFs
 * (G = 1 on patch j); n+1..2n U-type MBFs (G = -sigma beta_f on patch j);
 * sigma = +1 on the lower side of an interface, -1 on the upper.
 *
 * *out: NULL to create a handle; or a handle from an earlier call with the
 * same grid, walls, pin, partition, interface space and options, which is
 * rebuilt in place for the new coefficient arrays without any allocation.
 * Errors: MRCM_EINVAL (arguments, non-positive or non-finite K),
 * MRCM_EUNSUPPORTED (a local bandwidth or right-hand-side count beyond the
 * kernels' limits), MRCM_ENOTSPD (subdomain id in mrcm_last_error),
 * MRCM_ENOCONV (FP32_IR), MRCM_ENOMEM, MRCM_EHIP.  On error a handle created
 * by this call is destroyed and *out is left unchanged.
 */
mrcm_status mrcm_build_mbfs(const mrcm_problem *problem, const mrcm_partition *partition,
                            const mrcm_iface_space *iface, const mrcm_options *options,
                            void *stream, mrcm_mbfs **out);

/*
 * Interface assembly (Algorithm 2, "Assembly"; eqs. (2.18)-(2.22)).  For patch
 * i shared by subdomains s (two of them):
 *   P-row: sum_s sum_{j in I^s} (F^s[i,P_j] pi^p_j + F^s[i,U_j] pi^u_j) = -sum_s F^s[i,0]
 *   U-row: sum_s sigma^s_i sum_j (Fb^s[i,P_j] pi^p_j + Fb^s[i,U_j] pi^u_j)
 *          - (sum_s sum_{f in i} A_f beta^s_f) pi^u_i = -sum_s sigma^s_i Fb^s[i,0]
 * Each entry receives at most two contributions, so the result is bitwise
 * reproducible.  The entries go straight into the frontal matrices of the
 * multifrontal factorisation (nested dissection of the patch graph: planes
 * of interfaces cut boxes of subdomains in two, recursively); the first call
 * on a handle builds that plan and allocates the fronts.  *out: NULL to
 * create, or a handle from an earlier call on the same mbfs handle (reused
 * without allocation).  Errors: MRCM_EUNSUPPORTED (a front beyond the
 * sweep kernels' shared memory), MRCM_ENOMEM, MRCM_EHIP.
 */
mrcm_status mrcm_assemble_interface(const mrcm_mbfs *mbfs, void *stream, mrcm_interface **out);

/* Interface solvers (InterfaceSolver of Algorithm 2; the paper factorises
 * the interface system with a direct sparse LU). */
enum { MRCM_IFACE_AUTO = 0,         /* the multifrontal form */
       MRCM_IFACE_BAND = 1,         /* band LDL^T after a reverse Cuthill-McKee order (allocates its band,
                                       2 n (2w+1) doubles, on first use; systems up to a few 10^5 unknowns) */
       MRCM_IFACE_MULTIFRONTAL = 2  /* multifrontal LDL^T on the nested-dissection tree */ };

/*
 * Solves A^int X = b^int in FP64.  With s = -1 on the pressure rows and +1 on
 * the velocity rows, diag(s) A^int is symmetric quasi-definite, so it has an
 * LDL^T factorisation in any symmetric order without pivoting; the factor
 * then serves iterative refinement against the assembled (unfactored) system:
 * X += (LDL^T)^-1 diag(s) (b - A X).
 *  method      MRCM_IFACE_*.
 *  rtol        > 0: refine until ||b - A X|| / ||b|| <= rtol or max_refine
 *              steps (one stream synchronisation per step);
 *              0: exactly max_refine steps, no synchronisation (capturable).
 *  max_refine  0 .. 20.
 *  X [dev]     2*N_V doubles, pi^p then pi^u.
 *  iters [host] or NULL: refinement steps taken.
 *  rel_residual [host] or NULL: ||b - A X|| / ||b|| of the returned X (one
 *              more residual and a synchronisation).
 * Errors: MRCM_EINVAL, MRCM_ESINGULAR (zero pivot), MRCM_ENOMEM (band form),
 * MRCM_EHIP.
 */
mrcm_status mrcm_solve_interface(mrcm_interface *iface, int32_t method, double rtol, int32_t max_refine,
                                 void *stream, double *X, int32_t *iters, double *rel_residual);

/* Sizes of the interface system and its multifrontal factorisation, and the
 * last solve's method, refinement steps and residual (-1 if not computed). */
typedef struct {
  int32_t n;               /* unknowns, 2 N_V */
  int32_t nodes;           /* separators of the nested dissection */
  int32_t levels;          /* tree height */
  int32_t max_front;       /* largest frontal matrix */
  int64_t front_bytes;     /* all fronts (FP64, f x f each) */
  double factor_flops;     /* sum over separator pivots of (f - k - 1)^2 */
  int32_t factor_launches; /* panel-step launches of the factorisation */
  int32_t bandwidth;       /* band form: half bandwidth after the RCM order, or -1 if not built */
  int64_t device_bytes;    /* device memory held by the handle */
  int32_t method;          /* MRCM_IFACE_BAND or MRCM_IFACE_MULTIFRONTAL */
  int32_t refine_iters;
  double rel_residual;
} mrcm_interface_info;
mrcm_status mrcm_interface_query(const mrcm_interface *iface, mrcm_interface_info *info /* [host] */);

/*
 * Loop 2 of Algorithm 2 by the combination (2.23): p^l = X_l [1, pi^p_{I^l}, pi^u_{I^l}].
 * Velocities (per cell, outward normal, own side) follow (2.12) inside a
 * subdomain, Q_f / A_d = T_f (p_c - G_f(pi)) / A_d with
 * G_f = pi^p_i - sigma beta_f pi^u_i on Gamma, and the wall rules on the walls.
 * X [dev] 2*N_V interface unknowns; p [dev] N; U [dev] 6*N, face-major
 * (U[f*N + c]).
 */
mrcm_status mrcm_reconstruct(const mrcm_mbfs *mbfs, const double *X, void *stream,
                             double *p, double *U);

/*
 * The "Mean" post-processing of a multiscale velocity (Sec. 6, eq.
 * (locprob_submean)), which makes it conservative cell by cell for a
 * transport step.  On every fine face of Gamma between cells c and n the
 * normal velocity becomes the mean of the two sides' values, outward from c
 * (U[f][c] - U[f^1][n]) / 2.  Each subdomain then solves its Neumann problem:
 * the TPFA operator of (2.10) on its own cell pairs, the source q, and as
 * boundary data those Gamma velocities and, on the domain walls, U itself.
 * The problem fixes the pressure only up to a constant: the subdomain's
 * lowest-corner cell is set to zero (its row becomes the identity; the
 * multiscale solution's weak flux continuity leaves that row's balance with a
 * defect at the rounding of the interface solve).  Output: pt, the Neumann
 * pressures in that gauge, and Ut, the velocity from pt on faces inside a
 * subdomain and from the data on Gamma and the walls.
 * Arithmetic: the FP64 band Cholesky of the Jacobi-scaled local matrices and
 * one FP64 refinement sweep, whatever the handle's precision; the factors go
 * to a scratch of at most 8 GiB (less when the environment variable
 * MRCM_MEAN_SCRATCH_BYTES, read at the first call on a handle, asks for less)
 * that holds a chunk of subdomains at a time.  The chunking does not change
 * the result.
 * U [dev] 6*N face-major (the layout mrcm_reconstruct writes); pt [dev] N;
 * Ut [dev] 6*N, which must not overlap U.  The build's permeability and
 * source arrays must still be valid.  The first call allocates 64 bytes per
 * cell and the scratch, kept until mrcm_mbfs_destroy, and is not allowed
 * under graph capture.  Synchronises the stream (it reads the factor's
 * status).  Returns MRCM_EUNSUPPORTED when the largest subdomain's band
 * exceeds 112, MRCM_ENOTSPD on a non-positive pivot.
 */
mrcm_status mrcm_postprocess_mean(const mrcm_mbfs *mbfs, const double *U, void *stream, double *pt,
                                  double *Ut);

/*
 * Two-phase saturation step (IMPES, Sec. 5 and the implementation section:
 * eqs. (transporte_discreto), (flux_disc_up), (CFL)).  Water saturation S,
 * viscosity ratio M = mu_o / mu_w, fractional flow
 * phi(S) = M S^2 / (M S^2 + (1 - S)^2), total mobility
 * lambda(S) = S^2 / mu_w + (1 - S)^2 / mu_o.  Grid of nx x ny x nz cells of
 * hx x hy x hz, cells x fastest; porosity absorbed into time, as the paper does.
 */
typedef struct {
  int32_t nx, ny, nz;
  double hx, hy, hz;
  double mu_w, mu_o;   /* water and oil viscosities, > 0 */
} mrcm_twophase;

/*
 * One saturation step.  With U[6][N] the outward normal velocities per cell
 * and face (-x, +x, .., +z; face-major U[f*N + c], the layout mrcm_reconstruct
 * and mrcm_postprocess_mean write), the upwind update with the divergence
 * compensation reads
 *   S'_c = S_c - dt sum_f (phi_f - phi(S_c)) U[f][c] / h_d(f),
 * phi_f = phi(S_c) on an outflow face (U >= 0), the neighbour's phi on an
 * inflow face, and 1 (water) for an inflow across a domain wall; an injector
 * (q_c > 0) adds dt q_c (1 - phi(S_c)) / V.  (The printed update's signs and
 * its divergence term without the 1/h factors are read this way; the term
 * phi_c div u it removes includes div u = q / V in a well cell, which the
 * injector term restores for the water injected.)
 * U, S [dev] 6*N and N; q [dev] N total source rates (volume per time) or
 * NULL; dt [dev] one double, the step (mrcm_transport_dt writes it); S_out
 * [dev] N, which must not overlap S.  dt must be finite (an infinite one
 * gives NaN where a face velocity is zero).
 */
mrcm_status mrcm_transport_step(const mrcm_twophase *tp /* [host] */, const double *U, const double *q,
                                const double *S, const double *dt, void *stream, double *S_out);

/*
 * The saturation step for the current S and U under eq. (CFL), into dt
 * [dev] (one double): dt = min(dt_max, cfl min(hx, hy, hz) / M) with
 * M = max_c |phi'(S_c)| max_f |U[f][c]|, and dt = dt_max when M is zero.
 * dt_max is the loop's own step (an input of the IMPES loop, which the bound
 * may shorten); +inf leaves the bound alone.  The bound sees the face flows
 * only: from an all-oil state (phi' = 0 everywhere) it is infinite, and an
 * injector's own rate is bounded by dt_max (dt q / V <= 1 - S keeps its
 * cell within [0, 1]).  cfl = 1 is the printed bound; cfl <= 1/6 keeps S
 * within [0, 1] for any inflow pattern (six faces).  The value stays on the
 * device, so that steps chain without a synchronisation; dt's eight bytes
 * also serve as the reduction's accumulator.  cfl > 0 and finite, dt_max > 0.
 */
mrcm_status mrcm_transport_dt(const mrcm_twophase *tp /* [host] */, const double *U, const double *S, double cfl,
                              double dt_max, void *stream, double *dt);

/*
 * One saturation step (as mrcm_transport_step) and the next step under the
 * same velocity (as mrcm_transport_dt on S_out, with cfl and dt_max) in one
 * pass over U and S: the inner loop of the IMPES run, where the velocity is
 * held for C steps between Darcy solves.  dt [dev] the step to take,
 * dt_next [dev] the next one (must not be dt; ping-pong two doubles).
 * S_out must not overlap S.  marks [dev] or NULL: the marks of q made by
 * mrcm_transport_mark_sources (q is then read only in the marked parts of
 * the grid; 8 of the step's 72 bytes per cell otherwise).  Results equal the
 * two separate calls bitwise, with or without the marks.
 */
mrcm_status mrcm_transport_advance(const mrcm_twophase *tp /* [host] */, const double *U, const double *q,
                                   const void *marks, const double *S, const double *dt, double cfl, double dt_max,
                                   void *stream, double *S_out, double *dt_next);

/*
 * The marks of the cells where q is nonzero, for mrcm_transport_advance:
 * one byte per tile of the step (64 cells along x by 4 rows by up to 32
 * planes), nonzero where the tile holds a source.  They stay valid while q
 * does (the sources of an IMPES run usually hold for the whole run).
 * mrcm_transport_marks_bytes: the size of marks for the grid (0 on a bad
 * descriptor).  marks [dev]: that many bytes, written.
 */
int64_t mrcm_transport_marks_bytes(const mrcm_twophase *tp /* [host] */);
mrcm_status mrcm_transport_mark_sources(const mrcm_twophase *tp /* [host] */, const double *q, void *stream,
                                        void *marks);

/*
 * The permeability of a Darcy solve of the two-phase run: K lambda(S) per
 * cell (eq. sec2:darcy).  S, kx, ky, kz [dev] N in; kx_out, ky_out, kz_out
 * [dev] N out (may be the inputs themselves).
 */
mrcm_status mrcm_mobility_scale(const mrcm_twophase *tp /* [host] */, const double *S, const double *kx,
                                const double *ky, const double *kz, void *stream, double *kx_out, double *ky_out,
                                double *kz_out);

/*
 * The IMPES loop of the implementation section's overview algorithm: with
 * t = 0 and n = 0, while t <= t_end (and n < max_steps when that is > 0):
 * every skip-th saturation step (n mod C = 0, C the skipping constant) a
 * Darcy solve under the current saturation -- the permeability scaled by
 * lambda(S) (mrcm_mobility_scale), the MBFs rebuilt in place
 * (mrcm_build_mbfs), the interface assembled and solved (multifrontal,
 * `refine` refinement steps), the velocity reconstructed and post-processed
 * by the Mean method (mrcm_postprocess_mean), and the CFL step of that
 * velocity (mrcm_transport_dt) -- then one saturation step under the held
 * velocity (mrcm_transport_advance, which also gives the next step), t += dt,
 * n += 1.  The steps run in batches of up to 64 with their dt logged on the
 * device and read back once per batch (one synchronisation per batch); a run
 * that ends inside a batch is taken back to the batch's start and redone to
 * the step where it ends, with the same result as stepping one at a time.
 * problem, partition, iface, options: as for mrcm_build_mbfs; problem->kx,
 * ky, kz are the permeability K without the mobility, problem->q the sources
 * of both the Darcy solves and the saturation steps.  tp: the same grid and
 * cell sizes, and the viscosities.  S [dev] N: the initial saturation in,
 * the final one out.  stats [host] or NULL.
 * Errors: as the calls above; MRCM_EINVAL also for a step that is not finite
 * (nothing moves under the bound and dt_max is +inf), with S left at the
 * last finite state.  The library allocates the loop's buffers (about 19
 * doubles per cell, beside the MBF handle's) and frees them before it
 * returns; the handles it creates are destroyed too.
 */
typedef struct {
  int32_t skip;        /* C >= 1: saturation steps per Darcy solve */
  int32_t max_steps;   /* stop after this many saturation steps; 0: no cap */
  double t_end;        /* T: run while t <= T (+inf with max_steps > 0) */
  double cfl;          /* the factor of eq. (CFL), > 0 */
  double dt_max;       /* the loop's own step Dt_s (> 0; +inf: the bound alone) */
  int32_t refine;      /* interface refinement steps per Darcy solve, 0 .. 20 */
} mrcm_impes_options;

typedef struct {
  int32_t darcy_solves;   /* Darcy solves made */
  int32_t steps;          /* saturation steps taken */
  double t;               /* time reached */
  double ms_darcy;        /* device time of the mobility, MBF build, interface and reconstruction */
  double ms_darcy_first;  /* the part of ms_darcy spent in the first solve (which creates the handles) */
  double ms_mean;         /* device time of the Mean post-processing and the first CFL steps */
  double ms_transport;    /* device time of the saturation steps */
} mrcm_impes_stats;

mrcm_status mrcm_impes_run(const mrcm_problem *problem, const mrcm_partition *partition,
                           const mrcm_iface_space *iface, const mrcm_options *options,
                           const mrcm_twophase *tp /* [host] */, const mrcm_impes_options *io /* [host] */,
                           void *stream, double *S, mrcm_impes_stats *stats /* [host] */);

/*
 * Sizes and counts of a built handle.  n_patch counts the patches of the
 * interface space (each carries two unknowns, so 2 n_patch is the interface
 * system's size, the N_Gamma of eq. (2.24) for one patch per interface);
 * n_mbfs = sum over subdomains of 2|I^l| and n_rhs = n_mbfs + n_sub: one
 * P-type and one U-type MBF per patch of the subdomain, eq. (2.25), plus the
 * particular problem, eq. (2.26), as counted in Sec. 2.2.3 (13 for an
 * interior subdomain with one patch per face).  factor_flops and solve_flops
 * are the band algorithms' own operation counts; ir_* and pcg_* describe the
 * last build.
 */
mrcm_status mrcm_query(const mrcm_mbfs *mbfs, mrcm_info *info /* [host] */);
mrcm_status mrcm_get_subdomain(const mrcm_mbfs *mbfs, int32_t l, mrcm_subdomain_info *info /* [host] */);

/* Copies for tests and tools (synchronous; [host] outputs).
 *  mrcm_copy_mbfs:    X_l, row-major [n_cells][n_rhs] in the local row ordering.
 *  mrcm_copy_flux:    F and Fb [n_patch][n_rhs], SAb [n_patch] (sum A beta per patch).
 *  mrcm_copy_factor:  Cholesky factor L of the Jacobi-scaled local matrix
 *                     D^-1/2 A^H_l D^-1/2 (D its diagonal) in the local row order,
 *                     by column, [n_cells][band+1] with entry (j, t) = L[j+t][j],
 *                     converted to double.
 */
mrcm_status mrcm_copy_mbfs(const mrcm_mbfs *mbfs, int32_t l, double *X);
mrcm_status mrcm_copy_flux(const mrcm_mbfs *mbfs, int32_t l, double *F, double *Fb, double *SAb);
mrcm_status mrcm_copy_factor(const mrcm_mbfs *mbfs, int32_t l, double *Lband);

/* Interface system introspection: n = 2*N_V and the band form's half
 * bandwidth (-1 until the band form is used).  mrcm_copy_interface: the
 * assembled (unfactored) matrix as dense row-major [n][n] in the natural
 * unknown order (pi^p then pi^u), and b [n], formed on the device from the
 * flux blocks exactly as the solvers see them (allocates n^2 doubles for the
 * duration of the call). */
mrcm_status mrcm_interface_dims(const mrcm_interface *iface, int32_t *n, int32_t *bandwidth);
mrcm_status mrcm_copy_interface(const mrcm_interface *iface, double *A, double *b);

/*
 * Stage profiling with HIP events recorded on the caller's stream (tracing
 * subsystem; off by default).  While enabled, every call records an event
 * pair around each stage and accumulates the elapsed milliseconds and the
 * number of occurrences in a process-wide table, resolved when the call has
 * synchronised.  Stages, each one kernel launch unless noted: coefficients,
 * local factorisation, right-hand sides of (2.25)/(2.26), the local band
 * solves, the FP64 residuals of refinement (a fill, the residual and, in
 * FP32, the convergence check), the correction solves of refinement,
 * Gamma-flux reduction, interface assembly (several kernels), interface
 * LDL^T factorisation with the forward substitution (one step kernel per
 * 16-column block), interface backward sweeps (two kernels per 128 unknowns)
 * and refinement, reconstruction (two kernels).
 * FP64 form with refinement and FP32 form, when the solve work exceeds one
 * round of resident workgroups: 'solve' is the first solve of group 0 (the
 * first round's subdomains); 'refine' covers the rest -- group 1's first
 * solve and both groups' residuals and corrections (FP32: the first
 * min(3, ir_max_iter) sweeps), group 0's on a second stream that joins the
 * caller's stream at the end.  'residual' stays empty in the FP64 form; in
 * the FP32 form it holds the convergence checks and any further sweeps.
 * PCG: 'pcg' is the conjugate-gradient kernel and the read-back of its
 * convergence flags; 'fallback' the band Cholesky and direct solves of the
 * subdomains it left (factor and solve stages stay empty).  'solve_rest' is
 * the single launch of group 1's first solve, inside 'refine'.  Interface
 * stages: 'assemble' the scatter into the fronts (band form: into the band),
 * 'lu' the factorisation, 'sweep' the solves and refinement steps.  'mean'
 * is the whole of mrcm_postprocess_mean.
 */
enum { MRCM_STAGE_COEF = 0, MRCM_STAGE_FACTOR, MRCM_STAGE_RHS, MRCM_STAGE_SOLVE,
       MRCM_STAGE_RESIDUAL, MRCM_STAGE_REFINE, MRCM_STAGE_FLUX, MRCM_STAGE_ASSEMBLE,
       MRCM_STAGE_LU, MRCM_STAGE_SWEEP, MRCM_STAGE_RECONSTRUCT, MRCM_STAGE_PCG,
       MRCM_STAGE_FALLBACK, MRCM_STAGE_SOLVE_REST, MRCM_STAGE_MEAN, MRCM_STAGE_TRANSPORT, MRCM_STAGE_COUNT };
typedef struct {
  double ms[16];        /* accumulated milliseconds per stage */
  int64_t count[16];    /* occurrences per stage */
} mrcm_profile;
void mrcm_profile_enable(int32_t on);
void mrcm_profile_reset(void);
mrcm_status mrcm_profile_get(mrcm_profile *out /* [host] */);

/*
 * Orchestration (Algorithm 2 as one unit of work): the whole step
 * mrcm_build_mbfs -> mrcm_assemble_interface -> mrcm_solve_interface ->
 * mrcm_reconstruct recorded once into a HIP graph by stream capture, then
 * replayed with one launch.
 *  Requirements: precision MRCM_FP64 (the other forms take host decisions
 *  between kernels); mbfs and iface already built for this configuration
 *  (the capture rebuilds in place and allocates nothing); stream not the
 *  null stream.  The graph keeps the addresses of the problem's arrays
 *  (kx, ky, kz, q, wall values) and of X, p and U: a replay reads the
 *  arrays' current contents, so a new field is copied into the same buffers.
 *  mrcm_graph_launch enqueues one replay (asynchronous).  Errors the kernels
 *  flag (invalid permeability, non-positive local pivot, zero interface
 *  pivot) are read by mrcm_graph_check, which synchronises the stream.
 *  The handles must outlive the graph; calls that overlap a replay on the
 *  same handles race.
 */
/*
 * Autotuner (orchestration, Algorithm 2 as a whole): times mrcm_build_mbfs on
 * the given problem for candidate values of solve_tiles and solve_group, then
 * the other launch_mode with the winners (each candidate on a handle of its
 * own: one untimed and three timed builds, synchronised, the fastest
 * counted), then, with the winning values and when
 * the problem has interface unknowns, the interface assembly and solve
 * (mrcm_assemble_interface + mrcm_solve_interface, no refinement) for
 * iface_panel 1, 2 and 4.  Writes into *best a copy of *base with the fastest
 * values; a candidate replaces the current choice only when it is at least
 * 2% faster, so that near-ties keep base's values.  *best_ms and *rule_ms
 * (either may be NULL): the fastest build and that of base's own pair.
 * Allocates and frees one handle per candidate.
 */
mrcm_status mrcm_autotune(const mrcm_problem *problem, const mrcm_partition *partition,
                          const mrcm_iface_space *iface_space, const mrcm_options *base, void *stream,
                          mrcm_options *best, double *best_ms, double *rule_ms);

/*
 * mrcm_autotune with a per-shape cache in the text file cache_path [host]
 * (created when missing; one line per entry: "mrcm-tune-2", the key, then
 * solve_tiles, solve_group, iface_panel, launch_mode, best_ms, rule_ms).  The key is a
 * 64-bit FNV-1a hash of what the tuned values depend on: grid and cell
 * sizes, partition cuts, interface splits, wall types, precision, beta_mode,
 * keep and the device's architecture name and compute-unit count -- not the
 * coefficient values.  On a hit *best is *base with the cached values and no
 * kernel runs; on a miss mrcm_autotune runs and its result is appended.
 * *from_cache [host] (may be NULL): 1 on a hit, else 0.  An unreadable or
 * unwritable file is an error (MRCM_EINVAL); malformed lines are skipped.
 */
mrcm_status mrcm_autotune_cached(const mrcm_problem *problem, const mrcm_partition *partition,
                                 const mrcm_iface_space *iface_space, const mrcm_options *base, void *stream,
                                 const char *cache_path, mrcm_options *best, double *best_ms, double *rule_ms,
                                 int32_t *from_cache);

typedef struct mrcm_graph mrcm_graph;
mrcm_status mrcm_graph_capture(const mrcm_problem *problem, const mrcm_partition *partition,
                               const mrcm_iface_space *iface_space, const mrcm_options *options,
                               mrcm_mbfs *mbfs, mrcm_interface *iface, int32_t refine, double *X, double *p,
                               double *U, void *stream, mrcm_graph **out);
mrcm_status mrcm_graph_launch(mrcm_graph *graph, void *stream);
mrcm_status mrcm_graph_check(mrcm_graph *graph, void *stream);
void mrcm_graph_destroy(mrcm_graph *graph);

void mrcm_mbfs_destroy(mrcm_mbfs *mbfs);
void mrcm_interface_destroy(mrcm_interface *iface);
const char *mrcm_status_string(mrcm_status status);
const char *mrcm_last_error(void);   /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* MRCM_H */
