/*
 * pawfe.h -- C ABI of the MI355X PAW-FE residual-based Chebyshev filter.
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the hot path
 * of the finite-element PAW eigensolver: the FE-discretized PAW operators
 * H, S and the approximate inverse overlap Sinv_hat, the residual-based
 * Chebyshev filtered subspace (Algorithm 2, "R-ChFSI"), the Rayleigh-Ritz
 * step that consumes it (Algorithm 1, steps 4-6), the residual norms of the
 * eigen-residual check, and the gradient of the band energy with respect
 * to the effective potential and the PAW coupling Delta_H.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh      periodic orthorhombic box [0,Lx)x[0,Ly)x[0,Lz), nx*ny*nz
 *           uniform hexahedral cells, C0 Lagrange elements of degree p on
 *           Gauss-Lobatto-Legendre nodes (FE discretization section).
 *           cell e = i + nx*(j + ny*k); local node l = a + np*(b + np*c),
 *           np = p+1, a along x; periodic DOF I = gx + Gx*(gy + Gy*gz),
 *           gx = (i*p + a) mod (nx*p), Gx = nx*p.  ndof M = nx*ny*nz*p^3.
 * Quadrature  nq Gauss-Legendre points per direction in every cell
 *           (eq. "Quadrature Integration"); q = qx + nq*(qy + nq*qz).
 * Multivectors  X[I*ld + n] for DOF I and column n (row-major, node-major,
 *           columns contiguous), ld >= number of columns.  FP64 unless the
 *           entry point says otherwise.  All multivectors are DEVICE memory
 *           owned by the caller.
 * Streams   every entry point enqueues its device work on the given
 *           hipStream_t (passed as void*; NULL = the null stream) and
 *           returns without synchronizing unless its comment says it does.
 * Errors    argument errors are returned before anything is enqueued; a
 *           HIP error returns PAWFE_EHIP.  No C++ exception crosses the
 *           ABI.  pawfe_last_error() gives a message for the calling thread.
 *           On a non-OK status the contents of output buffers are
 *           unspecified.
 * Ownership the caller owns every buffer it passes; the library owns only
 *           the operator's tables (allocated by pawfe_build_operator, freed
 *           by pawfe_destroy_operator) and a per-operator scratch area for
 *           the stand-alone applies.  Calls on one operator must not run
 *           concurrently (they share that scratch).
 */
#ifndef PAWFE_H
#define PAWFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pawfe_op pawfe_op;

typedef int32_t pawfe_status;
enum {
  PAWFE_OK = 0,
  PAWFE_EINVAL = 1,        /* bad argument (message in pawfe_last_error) */
  PAWFE_ENOMEM = 2,        /* device or host allocation failed */
  PAWFE_EHIP = 3,          /* a HIP runtime call failed */
  PAWFE_ENOTSPD = 4,       /* I + G Delta_S singular, or S^p not positive definite */
  PAWFE_ENONFINITE = 5,    /* NaN / Inf met where a finite value is required */
  PAWFE_EUNSUPPORTED = 6   /* valid request the library does not implement */
};

/* Arithmetic of the filter's recurrence part (mixed-precision paragraph of
 * the subspace-construction section).  PAWFE_FP64: everything FP64.
 * PAWFE_FP32: the residual recurrence R and the operator applies inside the
 * loop in FP32 with R stored in FP32, the Y*Lambda correction added in FP64
 * (Y kept in FP64), the final Sinv_hat R in FP32 promoted before + X Lambda.
 * PAWFE_BF16X3: as PAWFE_FP32 (FP32 data), but the cell contractions of the
 * local operator run as bf16x3 split products on the bf16 matrix cores
 * (x = hi + lo, two bf16 parts; a*b ~ lo_a hi_b + hi_a lo_b + hi_a hi_b with
 * FP32 accumulation; relative error ~2^-16 per product, the FP32 (TF32-like)
 * stand-in of the precision paragraph).  The projector reduction of real
 * operators runs the same way on the matrix cores; the projector add-back
 * stays FP32.  Accepted by the apply entry points, pawfe_apply_local,
 * pawfe_cheb_filter and its workspace query (not for graded meshes or the
 * GGA term: PAWFE_EUNSUPPORTED); data must be finite. */
enum { PAWFE_FP64 = 0, PAWFE_FP32 = 1, PAWFE_BF16X3 = 2 };

/* How G^a inside Delta_Sinv^a = (Delta_S^{a,-1} + G^a)^{-1} is formed
 * (eq. "Delta Sinv" and the cheaper variant after it):
 * EXACT_G: G^a = C^a^H M_D^{-1} C^a;  PP: G^a = <p_alpha | p_beta>. */
enum { PAWFE_SINV_EXACT_G = 0, PAWFE_SINV_PP = 1 };

/* Operator description.  All arrays are HOST memory, read during
 * pawfe_build_operator only.
 *
 * veff_q     [E][nq^3] effective potential (Ha) at the Gauss points
 *            (V_el + V_xc + V_z of eq. "FEM Ham entries").
 * pos        [natoms][3] atom positions (bohr), any real values (wrapped).
 * rcut       [natoms] augmentation radius r_c; needs r_c < min(L)/2.
 * nproj      [natoms] projectors per atom (1..32).
 * proj_l/proj_m/proj_sigma  per projector, atom after atom: channel
 *            p(d) = S_lm(d) exp(-|d|^2/(2 sigma^2)) (1 - |d|^2/r_c^2)^2 for
 *            |d| < r_c, else 0; S_lm the unnormalized real solid harmonics
 *            l=0: 1; l=1, m=-1,0,1: y, z, x; l=2, m=-2..2: xy, yz,
 *            3z^2-r^2, xz, x^2-y^2.
 * dH, dS     Delta_H^a and Delta_S^a (eq. "FE nonlocal contribution"),
 *            nproj[a]^2 row-major blocks, atom after atom.
 * kpoint     Cartesian Bloch vector k (bohr^-1); must be 0 unless is_complex;
 *            NaN/Inf gives PAWFE_ENONFINITE.
 * is_complex 1 for the complex (k-point) operator of the Bloch-periodic part
 *            u of psi = e^{i k.x} u: H_loc gains 1/2 |k|^2 M and the
 *            imaginary term -i sum_d k_d <N_I | d/dx_d N_J>, and C^a carries
 *            the phase e^{-i k.x} at every quadrature point x (x taken at the
 *            image next to the atom as given in pos, unwrapped), so G^{ab}
 *            and Delta_Sinv^a become complex Hermitian.  Every column
 *            argument of a complex operator is complex: (re, im) pairs of
 *            doubles (or floats at PAWFE_FP32), and ld and nvec count
 *            complex entries.  Any other value: PAWFE_EINVAL.
 * Supported (degree, nq): (2,4) (3,5) (4,6) (5,7) (6,8); 2 <= n_d <= 1024. */
typedef struct {
  int32_t ncell[3];
  double box[3];
  int32_t degree;
  int32_t nq1d;
  double kpoint[3];
  int32_t is_complex;
  const double* veff_q;
  int32_t natoms;
  const double* pos;
  const double* rcut;
  const int32_t* nproj;
  const int32_t* proj_l;
  const int32_t* proj_m;
  const double* proj_sigma;
  const double* dH;
  const double* dS;
  int32_t sinv_mode;
  /* Graded mesh (FE discretization section; the two-level meshes of the
   * figure "Finite-element meshes employed in PAW-FE"): NULL for uniform
   * cells of size box / ncell, else the cell boundaries of the three axes
   * one after another, ncell[d] + 1 values per axis, rising strictly from 0
   * to box[d].  Every cell is then an axis-aligned box of its own size (a
   * diagonal Jacobian per cell); the DOF map and colouring are unchanged.
   * HOST array, copied. */
  const double* xgrid;
  /* GGA term of eq. "FEM Ham entries": NULL, or V_GGA at the Gauss points,
   * HOST [E][3][nq^3] (component d of cell e at point q), copied.  With a
   * graded mesh or a GGA field the operator must be real (is_complex = 0)
   * and PAWFE_BF16X3 is not accepted (PAWFE_EUNSUPPORTED). */
  const double* vgga_q;
} pawfe_op_desc;

/* Builds the operator (FE discretization section; eq. "FEM Cmatrix" for the
 * projector matrices C^a; eqs. "Sinvapprox"/"Delta Sinv" for Sinv_hat):
 * DOF map, cell colouring, GLL/Gauss 1-D tables, V(q) W_q, per-atom
 * support (cells with a Gauss point strictly inside r_c of the minimum
 * image of the atom), C^a on the support nodes, lumped GLL mass M_D, the
 * block-sparse G^{ab} = C^a^H M_D^{-1} C^b for atoms sharing support nodes,
 * and Delta_Sinv^a = Delta_S^a (I + G^a Delta_S^a)^{-1}.  Host work, then
 * upload on `stream`; synchronizes the stream before returning.
 * *out receives the new operator (NULL on failure). */
pawfe_status pawfe_build_operator(const pawfe_op_desc* desc, void* stream, pawfe_op** out);

/* Frees the operator's device tables.  NULL is accepted. */
pawfe_status pawfe_destroy_operator(pawfe_op* op);

/* Sizes: ndof M, quadrature points E*nq^3, number of cell colours, total
 * projectors sum_a nproj[a], total support cells and support nodes summed
 * over atoms (sizes for pawfe_get_dofmap).  Any pointer may be NULL. */
pawfe_status pawfe_query(const pawfe_op* op, int64_t* ndof, int64_t* nquad, int32_t* ncolour,
                         int32_t* nproj_total, int64_t* nsupp_cells, int64_t* nsupp_nodes);

/* Copies the builder's integer outputs to HOST arrays (any may be NULL):
 * cell_dofs [E][np^3], cell_colour [E], supp_cell_off [natoms+1] and
 * supp_cells (sorted per atom), supp_node_off [natoms+1] and supp_nodes
 * (sorted unique DOFs of the support cells, per atom). */
pawfe_status pawfe_get_dofmap(const pawfe_op* op, int32_t* cell_dofs, int32_t* cell_colour,
                              int64_t* supp_cell_off, int64_t* supp_cells,
                              int64_t* supp_node_off, int64_t* supp_nodes);

/* Copies to the HOST array first_visit [E] the builder's first-visit bits
 * of the colour-ordered assembly that the filter's fused step uses: bit
 * ca + 3 cb + 9 cc of first_visit[e] is set when cell e is the cell of the
 * lowest colour among the cells sharing its local nodes of position class
 * (ca, cb, cc) (per axis 0: the low face, 1: inside, 2: the high face), so
 * that every DOF has exactly one first visit.  Integer data, compared
 * bit-exactly by the tests. */
pawfe_status pawfe_get_first_visit(const pawfe_op* op, uint32_t* first_visit);

/* Replaces V(q) (HOST array [E][nq^3]) / Delta_H (HOST, packed like desc.dH).
 * Enqueued on `stream`, synchronizes it.  Delta_Sinv does not depend on
 * either, so nothing else is rebuilt. */
pawfe_status pawfe_set_veff(pawfe_op* op, const double* veff_q, void* stream);
/* Replaces V_GGA (HOST array [E][3][nq^3]) of an operator built with one
 * (PAWFE_EINVAL otherwise).  Enqueued on `stream`, synchronizes it. */
pawfe_status pawfe_set_vgga(pawfe_op* op, const double* vgga_q, void* stream);
pawfe_status pawfe_set_dH(pawfe_op* op, const double* dH, void* stream);

/* Y = A X for nvec columns (FE discretization section; cell-matrix AX
 * product of the operator-action subsection):
 *   apply_H:    H X = H_loc X + sum_a C^a Delta_H^a C^a^H X
 *   apply_S:    S X = M X + sum_a C^a Delta_S^a C^a^H X   (consistent M)
 *   apply_Sinv: Sinv_hat X = M_D^{-1} X - sum_a M_D^{-1} C^a Delta_Sinv^a
 *               C^a^H M_D^{-1} X
 * X, Y device, [ndof][ld]; FP64 (prec = PAWFE_FP64) or FP32 (PAWFE_FP32);
 * complex operators: complex entries, (re, im) interleaved.
 * X and Y must not overlap. */
pawfe_status pawfe_apply_H(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                           int64_t nvec, int32_t prec, void* stream);
pawfe_status pawfe_apply_S(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                           int64_t nvec, int32_t prec, void* stream);

/* pawfe_apply_H for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, layouts and result as pawfe_apply_H, but it calls no
 * hipMalloc / hipFree or allocating library routine.  The projector scratch
 * (partial sums and coefficients) lives in a 64 MiB static device array of
 * the library, one per GPU, held from the library's load on that GPU until
 * the process ends; the columns are processed in chunks (at most 512 real
 * columns) sized to fit it.  Returns PAWFE_EINVAL when the operator's
 * scratch for a single column exceeds 64 MiB.  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialized by the caller. */
pawfe_status pawfe_apply_H_noalloc(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                   int64_t nvec, int32_t prec, void* stream);

pawfe_status pawfe_apply_Sinv(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                              int64_t nvec, int32_t prec, void* stream);

/* BF16 halo of a slab decomposition along z (Reduced precision
 * inter-processor communication paragraph and the BF16-communication
 * figure: partial sums on the node planes shared with a neighbouring
 * processor travel in BF16 and are cast back to FP32 and added by the
 * receiver).  A slab is the cell layers [kz0, kz1) (0 <= kz0 < kz1 <= nz,
 * kz1 - kz0 < nz: a slab spanning the whole periodic mesh shares no plane
 * with another one; PAWFE_EINVAL) of the periodic mesh; its shared node
 * planes are gz0 = kz0 p and gz1 = (kz1 p) mod (nz p).
 *   pack:   buf[t][i][n] = BF16 bits of Y[plane_t row i][n], rounded to
 *           nearest, ties to even (NaN stays NaN);
 *   unpack: Y[plane_t row i][n] += (float) buf[t][i][n]   (FP32 add)
 * Y: device FP32 [ndof][ldy] (complex operators: (re, im) pairs, nvec
 * complex columns); buf: device [2][Gx*Gy][nvec] uint16 (complex: 2 nvec),
 * plane gz0 first, a plane's nodes in DOF order (gy, gx row-major).  The
 * buffer is caller-owned; Y and buf must not overlap. */
pawfe_status pawfe_halo_pack_bf16(const pawfe_op* op, const float* Y, int64_t ldy, int64_t nvec, int32_t kz0,
                                  int32_t kz1, uint16_t* buf, void* stream);
pawfe_status pawfe_halo_unpack_bf16(const pawfe_op* op, const uint16_t* buf, int64_t nvec, int32_t kz0, int32_t kz1,
                                    float* Y, int64_t ldy, void* stream);

/* Local (cell) part only:  Y += alpha * A_loc X, A_loc = K + V (which = 0)
 * or the consistent mass M (which = 1): the cell-level step of the
 * operator-action subsection (extraction, per-cell contraction, assembly),
 * without the non-local PAW term.  One launch per cell colour.  Used to
 * time the dominant kernel in isolation.  Same layouts as pawfe_apply_H. */
pawfe_status pawfe_apply_local(const pawfe_op* op, int32_t which, const void* X, int64_t ldx, void* Y,
                               int64_t ldy, int64_t nvec, double alpha, int32_t prec, void* stream);

/* Local part of one Chebyshev step of the filter (Algorithm 2, step 4, as
 * the filter runs it in FP64 and FP32), exposed to time and test the fused
 * cell kernel on its own:
 *   RX[I][n] <- (-ac RY[I][n] - zz RX[I][n]) + a lamY[n] Y[I][n]
 *               + a (H_loc M_D^{-1} RY)[I][n]
 * with H_loc = K + V (+ the GGA term) the cell part of H (operator-action
 * subsection; no PAW term) and M_D the lumped GLL mass (approximation (i) of eq. "Delta
 * Sinv").  In the filter RY holds R_Y - sum_a C^a d_a, so M_D^{-1} RY is
 * the block T = Sinv_hat R_Y of the step; the projector terms are added by
 * the filter around this call.  One launch per cell colour; the first term
 * is applied at the first visit of each DOF.
 * Columns are real: nvec real columns; complex operators store (re, im)
 * pairs of a complex column next to each other (nvec even), with lamY
 * given per real column.  RY, RX: device [ndof][ld] in FP64 (prec
 * PAWFE_FP64) or FP32 (PAWFE_FP32), same leading dimension; Y: device
 * double [ndof][ldy]; lamY: device double [nvec].  a, ac, zz: the step's
 * scalars a, a c and zeta zeta'.  RX must not overlap RY, Y or lamY; all
 * buffers are caller-owned.  Errors: PAWFE_EINVAL (NULL buffer, leading
 * dimension below nvec, odd nvec on a complex operator, nvec above 2^29);
 * PAWFE_EUNSUPPORTED (PAWFE_BF16X3, or a degree / Gauss rule without a
 * compiled variant). */
pawfe_status pawfe_cheb_step_local(const pawfe_op* op, const void* RY, void* RX, int64_t ld, const double* Y,
                                   int64_t ldy, const double* lamY, double a, double ac, double zz, int64_t nvec,
                                   int32_t prec, void* stream);

/* Bytes of workspace pawfe_cheb_filter needs for blocks of `block` columns:
 * room for two block states when nvec > block (two blocks in flight), else
 * one.  Any whole number of block states (the query with nvec = block gives
 * one) is accepted by pawfe_cheb_filter: one runs the blocks one after
 * another, k > 1 keeps up to min(k, 4) blocks in flight (two was the
 * fastest on the paper's workload). */
pawfe_status pawfe_cheb_filter_workspace(const pawfe_op* op, int64_t nvec, int32_t block,
                                         int32_t prec, size_t* bytes);

/* Algorithm 2 (residual-based Chebyshev filtered subspace), applied to the
 * nvec columns in uncoupled blocks of `block` columns with one polynomial:
 * e = (bU-bW)/2, c = (bU+bW)/2, zeta_1 = e/(b0-c); Y = H X - S X Lambda;
 * R_Y = (zeta_1/e) Y; for theta = 2..degree the recurrence
 * R_X <- a H Sinv_hat R_Y - a c R_Y - zeta zeta' R_X + a Y Lambda_Y with
 * zeta' = 1/(2/zeta_1 - zeta), a = 2 zeta'/e, and the same recurrence on
 * the diagonal Lambda; output Xout = Sinv_hat R_Y + X Lambda_Y.
 * Xin, Xout: device FP64 [ndof][ld]; Xout may equal Xin (in place).
 * lambda_in: device FP64 [nvec] (estimates of the eigenvalues).
 * Requires b0 < bW < bU, degree >= 2, 1 <= block.  ws: device workspace of
 * at least one block state (pawfe_cheb_filter_workspace with nvec = block),
 * 256-byte aligned.  With room for k >= 2 block states and more than one
 * block, block b runs on internal stream b mod min(k, 4, blocks) of the
 * library (default priority; one set per device, shared by all operators,
 * created on first use and kept until the process ends), forked from and
 * joined back into `stream`, so that one block's projector and node kernels
 * overlap another block's cell kernel; the results are identical to the
 * one-stream order.  Filters of different operators issued on different
 * streams at the same time run their blocks one after another on those
 * shared streams. */
pawfe_status pawfe_cheb_filter(const pawfe_op* op, const void* Xin, int64_t ldx, void* Xout,
                               int64_t ldo, int64_t nvec, int32_t block, const double* lambda_in,
                               int32_t degree, double b0, double bW, double bU, int32_t prec,
                               void* ws, size_t ws_bytes, void* stream);

/* The filter with step 2 of Algorithm 2 (the residual R = H X - S X Lambda
 * of the input pairs) supplied by the caller instead of formed here: R is
 * device FP64 [ndof][ldr] (complex operators: complex128), read only, for
 * the same nvec columns as Xin and the same lambda_in -- for instance the
 * residual that pawfe_rayleigh_ritz_res leaves of the Ritz pairs it
 * returns, which a ChFSI iteration filters next.  The output is then
 * bit-identical to pawfe_cheb_filter's.  R must not overlap Xout.  Other
 * arguments, workspace and errors as pawfe_cheb_filter; ldr < nvec or a
 * NULL R gives PAWFE_EINVAL. */
pawfe_status pawfe_cheb_filter_res(const pawfe_op* op, const void* Xin, int64_t ldx, const void* R,
                                   int64_t ldr, void* Xout, int64_t ldo, int64_t nvec, int32_t block,
                                   const double* lambda_in, int32_t degree, double b0, double bW,
                                   double bU, int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace pawfe_rayleigh_ritz needs. */
pawfe_status pawfe_rayleigh_ritz_workspace(const pawfe_op* op, int64_t nvec, size_t* bytes);

/* Rayleigh-Ritz (Algorithm 1 steps 4-6), FP64 throughout:
 * H^p = X^H H X, S^p = X^H S X (lower triangles, then Hermitized), the
 * projected generalized eigenproblem H^p Q = S^p Q Lambda, the rotation
 * X <- X Q (in place), and resnorm[i] = ||H x_i - lambda_i S x_i||_2 (the
 * eigen-residual check).  X device FP64 [ndof][ldx]; lambda (ascending)
 * and resnorm: device FP64 [nvec].  The projected problem is reduced with
 * the Cholesky factor S^p = U^H U (U^-H H^p U^-1 z = lambda z, Q = U^-1 Z).
 * Returns PAWFE_ENOTSPD if S^p is not positive definite (a non-positive
 * pivot of that factor; X is left unrotated) and PAWFE_ENONFINITE if the
 * eigensolver does not converge.  Synchronizes the stream (it reads the
 * factor's and the solver's status).
 * sr_prec: PAWFE_FP64 (the rotation as one FP64 GEMM) or PAWFE_FP32 (the
 * mixed-precision subspace rotation of the Rayleigh-Ritz subsection:
 * X diag(Q) in FP64 plus fl32(X) fl32(Q_off) as an FP32 GEMM, Q_off = Q with
 * its diagonal -- the complex diagonal entries -- set to zero; the residual
 * norms are those of the rotated vectors).
 * Complex operators: X holds nvec complex columns; the projected problem is
 * complex Hermitian (H^p, S^p and Q complex), lambda and resnorm stay real,
 * one entry per complex column. */
pawfe_status pawfe_rayleigh_ritz(const pawfe_op* op, void* X, int64_t ldx, int64_t nvec,
                                 double* lambda, double* resnorm, int32_t sr_prec, void* ws,
                                 size_t ws_bytes, void* stream);

/* Rayleigh-Ritz as pawfe_rayleigh_ritz, also writing the residual of the
 * rotated pairs, R = H X - S X Lambda (the columns whose 2-norms are
 * resnorm), into R: device FP64 [ndof][ldr] (complex operators:
 * complex128), caller-owned, not overlapping X.  pawfe_cheb_filter_res then
 * takes it as the filter's step 2.  ldr < nvec or a NULL R gives
 * PAWFE_EINVAL; otherwise as pawfe_rayleigh_ritz. */
pawfe_status pawfe_rayleigh_ritz_res(const pawfe_op* op, void* X, int64_t ldx, int64_t nvec,
                                     double* lambda, double* resnorm, void* R, int64_t ldr,
                                     int32_t sr_prec, void* ws, size_t ws_bytes, void* stream);

/* Band energy E = sum_n occ_n x_n^H H x_n and its gradient (the density and
 * projector contractions of the FE governing equations):
 *   dE_dVq[e][q] = W_{e,q} sum_n occ_n |u_n(x_{e,q})|^2, u_n the FE field;
 *   dE_dDH       = per atom sum_n occ_n conj(P_n) P_n^T, P_n = C^a^H x_n,
 *                  packed like desc.dH (full-matrix gradient).
 * X device FP64; occ device FP64 [nvec] or NULL (all ones); E device FP64
 * scalar; dE_dVq device [E*nq^3]; dE_dDH device [sum nproj^2].  Any output
 * may be NULL.  Nothing cell-local is stored between cell batches.
 * Complex operators: X holds complex columns; E = sum_n occ_n x_n^H H x_n,
 * the density sums |u_n|^2, and dE_dDH = Re sum_n occ_n conj(P_n) P_n^T. */
pawfe_status pawfe_band_energy_grad(const pawfe_op* op, const void* X, int64_t ldx, int64_t nvec,
                                    const double* occ, double* E, double* dE_dVq, double* dE_dDH,
                                    void* stream);

/* k-step Lanczos on H Sinv_hat in the Sinv_hat inner product (bound
 * estimate of Algorithm 1 step 1), seeded start vector.  HOST outputs:
 * smallest and largest Ritz value and |beta_k|; an upper bound of the
 * spectrum is theta_max + |beta_k|.  Synchronizes the stream. */
pawfe_status pawfe_lanczos_bounds(const pawfe_op* op, int32_t k, uint64_t seed, double* theta_min,
                                  double* theta_max, double* beta_k, void* stream);

/* Bytes of workspace pawfe_chfsi_solve needs: the larger of the filter's
 * (two block states when nvec > block) and Rayleigh-Ritz's, plus the FP64
 * residual of the Ritz pairs (ndof x nvec, complex operators twice that)
 * that each Rayleigh-Ritz hands to the next filter pass. */
pawfe_status pawfe_chfsi_solve_workspace(const pawfe_op* op, int64_t nvec, int32_t block, int32_t prec,
                                         size_t* bytes);

/* Algorithm 1 run to convergence (the outer ChFSI loop, with the
 * residual-norm test of its last step): b_U = bU if bU > 0, else the
 * Lanczos estimate theta_max + |beta_k| (pawfe_lanczos_bounds with
 * lanczos_k steps, seed 1234); Rayleigh-Ritz of the start X; then, while
 * the largest residual norm of the lowest nwanted Ritz pairs (all when
 * nwanted = 0) exceeds tol and fewer than max_iter passes have run: one
 * filter pass in place (degree, block, prec; b_0 and b_W the lowest and
 * highest current Ritz values, lambda_in the Ritz values), started from the
 * residual the last Rayleigh-Ritz formed (pawfe_cheb_filter_res), and one
 * FP64 Rayleigh-Ritz (pawfe_rayleigh_ritz_res).  The ws pointer must be
 * 256-byte aligned.  X device FP64 [ndof][ldx] (complex
 * operators: complex columns), replaced by the Ritz vectors; lambda and
 * resnorm device FP64 [nvec] (the last Rayleigh-Ritz); *iterations (host,
 * may be NULL) receives the number of filter passes.  Not reaching tol
 * within max_iter is not an error (check resnorm).  Needs nvec >= 2.
 * Synchronizes the stream after every Rayleigh-Ritz (reads the residual
 * norms). */
pawfe_status pawfe_chfsi_solve(const pawfe_op* op, void* X, int64_t ldx, int64_t nvec, int64_t nwanted,
                               int32_t degree, int32_t block, int32_t prec, double bU, int32_t lanczos_k,
                               double tol, int32_t max_iter, double* lambda, double* resnorm,
                               int32_t* iterations, void* ws, size_t ws_bytes, void* stream);

/* ---- Batched filter over independent problems (HIP graph) ----------------
 *
 * Several independent problems of uneven size (different operators, column
 * counts, polynomial degrees and bounds; the sum over k-points or small
 * cells of the band-energy expression, FE governing equations section)
 * are filtered together: each job is one pawfe_cheb_filter call.  The batch
 * sorts the jobs by estimated cost (largest first), cuts them in that order
 * into groups of at most max_graph_launches kernel launches (at least one
 * job per group; <= 0: 16384), spreads each group's jobs over nstreams
 * streams by longest-processing-time-first, captures each group's
 * multi-stream schedule once into its own HIP graph, and replays the graphs
 * one after another.  The budget bounds the size and the longest dependency
 * chain of every graph.  Every pointer of every job is baked into the
 * graphs: a replay re-reads the current CONTENTS of Xin and lambda_in and
 * overwrites Xout.
 *
 * Column block sizes: a job with block <= 0 gets its block size from the
 * autotuner, which times the candidates {64, 128, 256} (those <= nvec, and
 * nvec itself when smaller) with a short degree-3 filter of that job on a
 * private stream and keeps the fastest.  nstreams <= 0 lets the autotuner
 * time the whole batch eagerly for 1, 2 and 4 streams and keep the fastest.
 * The autotuning runs (eager filters on the jobs' own buffers) happen
 * inside pawfe_batch_create; their outputs are overwritten by any replay.
 *
 * Real and complex (k-point) operators may be mixed in one batch; the
 * columns of a complex job are complex (as for pawfe_cheb_filter).
 */
typedef struct pawfe_batch pawfe_batch;

typedef struct {
  const pawfe_op* op;        /* operator of this problem (not owned) */
  const void* Xin;           /* device FP64 [ndof][ldx] */
  int64_t ldx;
  void* Xout;                /* device FP64 [ndof][ldo]; may equal Xin */
  int64_t ldo;
  int64_t nvec;              /* columns */
  int32_t block;             /* columns per filter block; <= 0: autotuned */
  const double* lambda_in;   /* device FP64 [nvec] */
  int32_t degree;            /* Chebyshev degree m >= 2 */
  double b0, bW, bU;         /* filter bounds, b0 < bW < bU */
} pawfe_filter_job;

/* Builds the batch: validates every job (as pawfe_cheb_filter), allocates
 * one workspace per job (device memory owned by the batch), autotunes,
 * captures and instantiates the graph.  `stream` is used for the tuning
 * runs and is synchronized before return.  prec: PAWFE_FP64 or PAWFE_FP32
 * (the recurrence precision of every job).  The operators must outlive the
 * batch and must not be used by other calls while the batch runs. */
pawfe_status pawfe_batch_create(const pawfe_filter_job* jobs, int32_t njobs, int32_t prec, int32_t nstreams,
                                int32_t max_graph_launches, void* stream, pawfe_batch** out);

/* Enqueues one replay (every captured graph, in order) on `stream`
 * (asynchronous). */
pawfe_status pawfe_batch_run(pawfe_batch* batch, void* stream);

/* Chosen schedule: number of streams, per-job block size and stream index
 * (host arrays of njobs entries), number of captured graphs.  Any pointer
 * may be NULL. */
pawfe_status pawfe_batch_query(const pawfe_batch* batch, int32_t* nstreams, int32_t* blocks,
                               int32_t* stream_of_job, int32_t* ngraphs);

/* Frees the graph, the streams and the workspaces (synchronizes first). */
void pawfe_batch_destroy(pawfe_batch* batch);

/* Timed tuning runs (block-size trials and stream-count trials) that
 * pawfe_batch_create spent on this batch: 0 when every decision came from
 * the tuning cache below or was fixed by the caller. */
pawfe_status pawfe_batch_tuning_runs(const pawfe_batch* batch, int32_t* ntimed);

/* Tuning cache of the batch autotuner: the decisions of pawfe_batch_create
 * (block size and cost estimate per job, stream count per batch), kept
 * process-wide and keyed by what they depend on (GPU architecture, the
 * operator's cells, degree, Gauss rule, atoms and projectors, real or
 * complex, graded / GGA, the job's column count, Chebyshev degree and the
 * precision).  pawfe_batch_create consults it and adds what it tunes.
 *   _save: writes the table to the text file `path` (through `path`.tmp,
 *          then renamed); first line "pawfe-tune-cache 1", then one entry
 *          per line "<key> <block or stream count> <cost ms>".
 *   _load: merges a file written by _save; PAWFE_EINVAL for a missing
 *          file, a wrong first line or a line that does not parse (the
 *          table is then unchanged).
 *   _clear: empties the table.  _size: number of entries.
 * Host only, no GPU call; thread-safe. */
pawfe_status pawfe_tune_cache_load(const char* path);
pawfe_status pawfe_tune_cache_save(const char* path);
pawfe_status pawfe_tune_cache_clear(void);
pawfe_status pawfe_tune_cache_size(int64_t* nentries);

/* Message for the last non-OK status on the calling thread ("" if none). */
const char* pawfe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PAWFE_H */
