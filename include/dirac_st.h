/*
 * dirac_st.h -- C ABI of the MI355X spacetime finite-element Dirac solver.
 *
 * Method: "A Spacetime Finite Elements Method to Solve the Dirac Equation"
 * (arXiv:2103.14588).  The library assembles the Galerkin operator of the
 * Dirac equation on tensor-product Q1 spacetime elements (Sec. 2.2, App. A),
 * removes the t = 0 test rows and moves the t = 0 columns to the right-hand
 * side (Sec. 2.1, eq. (dirac_weakIVP); Alg. 1 steps 3-5), and solves the
 * resulting unsymmetric complex system with restarted GMRES (Sec. 2.2,
 * Alg. 1 step 6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer owned by the caller, unless
 *   the comment says "host".  Sizes come from dirac_st_sizes() and
 *   dirac_st_workspace_bytes().  The only device allocation the library makes
 *   is a 4-byte stream-ordered counter inside dirac_st_assemble (freed before
 *   it returns).  Nothing is retained after a call returns.
 * Complex layout.  Interleaved (re, im); complex128 = two doubles, complex64 =
 *   two floats (the layout of torch.complex128 / torch.complex64).
 * Vector layout.  Node-major, spinor component fastest: entry (r, c) at r*nc + c
 *   with block row r = (tau - 1) * S + s, tau = 1..n_t the time node, S the
 *   number of spatial nodes and s = i_1 + n_1 (i_2 + n_2 i_3) the spatial node
 *   (axis 1 fastest).  The initial field psi0 uses the same layout over the
 *   S nodes of the t = 0 slice.
 * Matrix layout.  Block CSR: row_ptr[nrows + 1], col_idx[nnzb] (int32, columns
 *   ascending in each row), values [nnzb][nc][nc] row-major (entry (i, j) of a
 *   block multiplies component j of the column node into component i of the
 *   row node).
 * Streams.  `stream` is a hipStream_t passed as void*; NULL is the default
 *   stream.  dirac_st_assemble, dirac_st_spmv and dirac_st_pc_apply only enqueue
 *   work.  The solvers enqueue on `stream` and synchronise it (they read
 *   convergence estimates back to the host); they return when done.
 * Errors.  Every function returns an int: DIRAC_ST_OK (0), DIRAC_ST_NOT_CONVERGED
 *   (1, solution and statistics valid), or a negative code.  The message of the
 *   last failure on the calling thread is dirac_st_last_error().
 * Threads.  Calls are reentrant given distinct workspaces and output buffers.
 */
#ifndef DIRAC_ST_H
#define DIRAC_ST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DIRAC_ST_OK = 0,
  DIRAC_ST_NOT_CONVERGED = 1,
  DIRAC_ST_EINVAL = -1,      /* invalid argument or unsupported problem */
  DIRAC_ST_EHIP = -2,        /* a HIP runtime call failed */
  DIRAC_ST_EBREAKDOWN = -3,  /* NaN/Inf in the iteration (e.g. in b) */
  DIRAC_ST_ENOSPACE = -4     /* workspace smaller than dirac_st_workspace_bytes() */
};

/* Potential kinds (Sec. 4.3).  V depends on the first spatial coordinate x. */
enum {
  DIRAC_ST_V_NONE = 0,
  DIRAC_ST_V_STEP = 1,   /* V = v0 for x > x0 (strict), 0 otherwise */
  DIRAC_ST_V_SMOOTH = 2  /* V = v0/2 (1 + tanh((x - x0)/lw)) */
};

/* Preconditioners (applied on the right, so GMRES minimises the true residual). */
enum {
  DIRAC_ST_PC_NONE = 0,
  DIRAC_ST_PC_BLOCK_JACOBI = 1, /* inverse of each node's nc x nc diagonal block */
  DIRAC_ST_PC_SPECTRAL = 2,     /* exact inverse of the operator with V replaced by
                                   the constant opts.vbar (periodic uniform mesh) */
  DIRAC_ST_PC_LINE = 3,         /* exact inverse of the operator itself for every
                                   potential of the method (all depend on x_1 only):
                                   time eigenbasis, DFT over x_2, x_3, periodic
                                   block-tridiagonal solves along x_1; needs
                                   n_t <= 2048 and workspace for nc*nc*4 factors
                                   per node */
  DIRAC_ST_PC_TIME_SLABS = 4    /* time decomposition (the direction the paper's
                                   conclusion proposes, time-additive Schwarz),
                                   non-overlapping: opts.time_slabs equal slabs
                                   of time rows; on each slab the exact inverse
                                   of the same Galerkin problem posed on the
                                   slab's own time interval (first row: the
                                   field before the slab is taken as zero; last
                                   row: ends like the last row of [0, T]),
                                   solved like DIRAC_ST_PC_LINE.  time_slabs
                                   must divide n_t; 1 slab = DIRAC_ST_PC_LINE */
};

/* Problem: the spacetime box [0, len[0]] x [0, len[1]] x ... with n[0] time
 * elements and n[1..d] spatial elements per axis, periodic in space.
 *   d      spatial dimensions, 1..3 (1+1, 2+1, 3+1 of Sec. 4.1)
 *   nc     spinor components: 2 for d = 1, 2 and 4 for d = 3
 *   n      n[0] >= 1; n[1..d] >= 3
 *   m      mass (hbar = c = 1, Sec. 2.1)
 *   vkind, v0, x0, lw   scalar potential, see DIRAC_ST_V_*.  It enters the
 *          operator as the potential energy: i d_t -> i d_t - V, i.e. the
 *          block term -g^0 int V phi_j phi_i, integrated with 2-point
 *          Gauss-Legendre per axis.
 * Gamma matrices: 1+1 and 2+1 use g0 = diag(1, -1), g1 = [[0, 1], [-1, 0]]
 * (App. A), and for 2+1 g2 = [[0, -i], [-i, 0]]; 3+1 uses the Dirac
 * representation. */
typedef struct {
  int32_t d;
  int32_t nc;
  int32_t n[4];
  double len[4];
  double m;
  int32_t vkind;
  double v0, x0, lw;
} dirac_st_problem;

/* Assembled operator A = D_w22 (Sec. 2.1).  All arrays are caller-allocated
 * device memory sized from dirac_st_sizes().  val32, bjinv64 and bjinv32 may be
 * NULL (then they are not written and the features needing them are off). */
typedef struct {
  int32_t *row_ptr;     /* [nrows + 1] */
  int32_t *col_idx;     /* [nnzb] */
  void *val64;          /* [nnzb][nc][nc] complex128 */
  void *val32;          /* [nnzb][nc][nc] complex64, RNE rounding of val64 */
  void *bjinv64;        /* [nrows][nc][nc] complex128 inverses of diagonal blocks */
  void *bjinv32;        /* [nrows][nc][nc] complex64 */
  int64_t nrows, nnzb;  /* set by the caller from dirac_st_sizes() */
  int32_t nc;           /* set by dirac_st_assemble */
  int32_t singular_blocks; /* host, set by dirac_st_assemble when bjinv64 != NULL:
                              diagonal blocks whose 1-norm condition number
                              exceeds 1e12 (replaced by the identity) */
  dirac_st_problem prob;   /* set by dirac_st_assemble; the spectral
                              preconditioner reads the mesh from here */
} dirac_st_bsr;

typedef struct {
  int32_t restart;    /* m, Arnoldi steps per cycle (1..64) */
  int32_t max_it;     /* cap on the total number of Arnoldi steps */
  int32_t pc;         /* DIRAC_ST_PC_* */
  int32_t precision;  /* 64: complex128 GMRES.  32: complex64 inner cycles
                         (SpMV on val32, basis and preconditioner in complex64)
                         inside an FP64 refinement loop: every cycle starts from
                         the FP64 true residual b - A x (val64) and adds its
                         correction to x in FP64.  Givens rotations and the
                         Hessenberg solve are FP64 in both modes. */
  int32_t max_cycles; /* cap on restart cycles (refinement steps); 0 = no cap */
  double rtol;        /* stop when ||b - A x||_2 <= rtol ||b||_2 (true residual) */
  double inner_rtol;  /* precision 32: a cycle also ends when its estimated
                         residual falls below inner_rtol times its starting
                         residual (0 = run the full cycle) */
  double vbar;        /* constant potential of DIRAC_ST_PC_SPECTRAL */
  int32_t time_slabs; /* DIRAC_ST_PC_TIME_SLABS: number of time slabs (>= 1,
                         divides n_t); ignored by the other preconditioners */
  int32_t matrix_free; /* dirac_st_gmres / dirac_st_bicgstab: 1 applies the
                          operator from A->prob with the matrix-free stencil
                          (dirac_st_spmv_mf) instead of the stored blocks, in
                          every product and residual; the value arrays of A
                          are then not read and may be NULL (node-block
                          Jacobi still needs bjinv64/32).  0: stored blocks. */
} dirac_st_opts;

typedef struct {
  int32_t iters;        /* Arnoldi steps taken */
  int32_t cycles;       /* restart cycles (= refinement steps for precision 32) */
  int32_t converged;    /* 1 if the true relative residual <= rtol */
  int32_t singular_blocks;
  double relres;        /* true relative residual ||b - A x|| / ||b|| at exit (FP64) */
  double est;           /* last Arnoldi residual estimate / ||b|| */
  double ms;            /* wall time of the solve on the host clock */
  double *history;      /* host, optional (NULL): residual estimate / ||b|| after
                           each Arnoldi step, up to history_len entries */
  int32_t history_len;
  int32_t fallback;     /* dirac_st_fgmres_nn: 1 if the network was switched off
                           (non-finite output or a cycle that cut the residual by
                           less than 1%) and the base preconditioner finished */
} dirac_st_stats;

/* Learned preconditioner network (2+1D fields only): 3x3x3 convolutions over
 * the spacetime grid [tau][y][x] with channels 4 -> 16 -> 16 -> 16 -> 4 (real
 * and imaginary parts of the two spinor components), ReLU between layers,
 * periodic padding in space and zero padding in time.  bfloat16 weights and
 * activations, FP32 accumulation on the matrix cores; FP32 master parameters
 * and Adam state.  All arrays are caller-owned device memory. */
typedef struct {
  float *params;        /* [17332]: per layer W[27][cin][cout] then b[cout]; tap
                           (dt+1)*9 + (dy+1)*3 + (dx+1) */
  float *adam_m;        /* [17332] first moments (training only, else NULL) */
  float *adam_v;        /* [17332] second moments (training only, else NULL) */
  uint16_t *w16;        /* [17280] bf16 weights, written by dirac_st_nn_pack */
  uint16_t *wt16;       /* [17280] bf16 weights with flipped taps and swapped
                           channel order (backward pass), written by dirac_st_nn_pack */
  int32_t step;         /* host: Adam steps taken (incremented by train_step) */
  float out_gain;       /* host: fixed output gain g of the preconditioner term,
                           z += g s N(v / s); chosen at training time so that the
                           network's targets are O(1) (0 is read as 1) */
} dirac_st_nn;

/* Number of FP32 parameters of the network (17332). */
size_t dirac_st_nn_param_count(void);

/* Device workspace of the network on an nt x ny x nx grid (training != 0: the
 * forward-backward pass of dirac_st_nn_train_step / dirac_st_nn_backward). */
size_t dirac_st_nn_workspace_bytes(int32_t nt, int32_t ny, int32_t nx, int32_t training);

/* Refresh w16 and wt16 from params (round to nearest even). */
int dirac_st_nn_pack(const dirac_st_nn *net, void *stream);

/* out = N(in_scale * in).  in, out: [nt][ny][nx][4] FP32 (a complex64 field
 * [nt][ny][nx][2] has this layout). */
int dirac_st_nn_forward(const dirac_st_nn *net, int32_t nt, int32_t ny, int32_t nx, const float *in,
                        double in_scale, float *out, void *work, size_t work_bytes, void *stream);

/* grad = d/dparams of <dout, N(in_scale * in)> (dout rounded to bf16 first,
 * like the training step).  grad: [17332] FP32. */
int dirac_st_nn_backward(const dirac_st_nn *net, int32_t nt, int32_t ny, int32_t nx, const float *in,
                         double in_scale, const float *dout, float *grad, void *work,
                         size_t work_bytes, void *stream);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the loss
 * ||N(in) - target||^2 / ||target||^2, then dirac_st_nn_pack.  loss_out: device
 * double receiving the loss before the step (may be NULL). */
int dirac_st_nn_train_step(dirac_st_nn *net, int32_t nt, int32_t ny, int32_t nx, const float *in,
                           const float *target, float lr, double *loss_out, void *work,
                           size_t work_bytes, void *stream);

/* Flexible GMRES(m) (right preconditioning with the preconditioned vectors
 * Z stored, x += Z y) for a 2+1D operator.  The preconditioner is
 * z = M^{-1} v + g s N(v / s) with M the base preconditioner opts->pc, g = net->out_gain and
 * s = ||v|| / sqrt(n) (n complex entries); net == NULL drops the network term.
 * If the network produces NaN/Inf or a cycle cuts the residual by less than
 * 1%, the network is switched off for the rest of the solve
 * (stats->fallback = 1).  The network workspace is part of `work`
 * (dirac_st_workspace_bytes with flexible = 1).  Returns as dirac_st_gmres. */
int dirac_st_fgmres_nn(const dirac_st_bsr *A, const void *b, void *x, const dirac_st_nn *net,
                       const dirac_st_opts *opts, void *work, size_t work_bytes,
                       dirac_st_stats *stats, void *stream);

/* Message of the last error on the calling thread ("" if none). */
const char *dirac_st_last_error(void);

/* Host.  Number of block rows (unknown nodes, tau = 1..n_t) and stored blocks
 * of the assembled operator: a row holds 3^(d+1) blocks, 2*3^d in the first
 * and last time slice (3^d if n_t = 1).  Sec. 2.1-2.2. */
int dirac_st_sizes(const dirac_st_problem *prob, int64_t *nrows, int64_t *nnzb);

/* Assemble A = D_w22 into block CSR and the right-hand side b = -D_w21 psi0
 * (Sec. 2.1, eq. (dirac_weakIVP); Sec. 2.2 element summation; App. A element
 * matrices).  psi0: [S][nc] complex128 nodal values at t = 0 (may be NULL if
 * b is NULL).  b: [nrows][nc] complex128 (may be NULL).  Fills A->row_ptr,
 * col_idx, val64 and, when non-NULL, val32, bjinv64, bjinv32; sets A->nc,
 * A->prob and A->singular_blocks (synchronises the stream to read the
 * count when bjinv64 != NULL).  A->nrows and A->nnzb must equal
 * dirac_st_sizes(). */
int dirac_st_assemble(const dirac_st_problem *prob, const void *psi0, dirac_st_bsr *A, void *b,
                      void *stream);

/* y = A x (Sec. 2.2: the product inside GMRES).  prec 64: complex128 x, y and
 * val64; prec 32: complex64 x, y and val32.  x and y must not overlap.  A must
 * come from dirac_st_assemble: for 2x2 blocks the block addresses and columns
 * are computed from A->prob (the stencil of the assembled pattern) and
 * row_ptr / col_idx are not read; 4x4 blocks use them. */
int dirac_st_spmv(const dirac_st_bsr *A, int32_t prec, const void *x, void *y, void *stream);

/* y = A x without a stored matrix: the operator of problem p (the one
 * dirac_st_assemble builds, Sec. 2.1-2.2 and App. A, potential of Sec. 4.3)
 * applied as a sum of Kronecker products of 1D three-point stencils, one
 * thread per row node, x staged in LDS per tile for d <= 2.  Equal to
 * dirac_st_spmv on the assembled matrix up to rounding order.  x, y: device,
 * [nrows][nc] complex128 (prec 64) or complex64 (prec 32), not overlapping.
 * Enqueues on `stream`; DIRAC_ST_EINVAL for an invalid problem or arguments. */
int dirac_st_spmv_mf(const dirac_st_problem *p, int32_t prec, const void *x, void *y, void *stream);

/* b = -D_w21 psi0 (Sec. 2.1, eq. (dirac_weakIVP)) without a stored matrix:
 * the right-hand side dirac_st_assemble writes, from the same stencils.
 * psi0: device, [S][nc] complex128 (the t = 0 slice); b: device,
 * [nrows][nc] complex128, zero outside tau = 1.  Enqueues on `stream`. */
int dirac_st_rhs_mf(const dirac_st_problem *p, const void *psi0, void *b, void *stream);

/* z = M^{-1} v for the preconditioner opts->pc (DIRAC_ST_PC_*, not NONE) in
 * precision opts->precision (64: complex128, 32: complex64), with its
 * parameters opts->vbar / opts->time_slabs.  work: workspace of at least
 * dirac_st_workspace_bytes(A, opts, 0) bytes (the spectral, line and time-slab
 * preconditioners keep their factorisations there; the call sets them up and,
 * for the line and time-slab preconditioners, synchronises the stream). */
int dirac_st_pc_apply(const dirac_st_bsr *A, const dirac_st_opts *opts, const void *v, void *z,
                      void *work, size_t work_bytes, void *stream);

/* Bytes of device workspace needed by dirac_st_gmres (flexible = 0) or
 * dirac_st_fgmres_nn (flexible = 1) for these options: basis of restart+1
 * vectors in the working precision, partial sums, Hessenberg data,
 * preconditioner data; flexible adds the restart preconditioned vectors and,
 * for 2+1D operators, the network's inference workspace. */
size_t dirac_st_workspace_bytes(const dirac_st_bsr *A, const dirac_st_opts *opts, int32_t flexible);

/* Restarted GMRES(m) with right preconditioning (Sec. 2.2; Alg. 1 step 6):
 * two-pass classical Gram-Schmidt, complex Givens rotations, x += M^{-1} V y at
 * the end of each cycle, true residual recomputed in FP64 at every restart.
 * b: [nrows][nc] complex128.  x: [nrows][nc] complex128, initial guess on
 * entry, solution on exit.  stats: host, may be NULL.  Returns DIRAC_ST_OK,
 * DIRAC_ST_NOT_CONVERGED (max_it or max_cycles reached), or an error
 * (DIRAC_ST_EBREAKDOWN if NaN/Inf appears, e.g. from b).  work_bytes: at least
 * dirac_st_workspace_bytes(A, opts, 0); with dirac_st_workspace_bytes(A, opts, 1)
 * or more (and a preconditioner) the preconditioned vectors are kept and the
 * end-of-cycle update x += Z y needs no second preconditioner application. */
int dirac_st_gmres(const dirac_st_bsr *A, const void *b, void *x, const dirac_st_opts *opts,
                   void *work, size_t work_bytes, dirac_st_stats *stats, void *stream);

/* Bytes of device workspace needed by dirac_st_bicgstab for these options:
 * eight complex128 vectors, partial sums, scalars, preconditioner data.
 * Returns 0 for an invalid matrix. */
size_t dirac_st_bicgstab_workspace_bytes(const dirac_st_bsr *A, const dirac_st_opts *opts);

/* BiCGSTAB, the second Krylov solver of the paper's parallel runs (Sec. 4.4,
 * Tables 1-3; van der Vorst's algorithm), right-preconditioned so that r is
 * the residual of A x = b, in complex128 (opts->precision must be 64).  Per
 * iteration two products with A and two preconditioner applications; the
 * scalars stay on the device and the host reads 16 bytes per iteration.  The
 * stop test uses the updated residual; when it passes, the FP64 true
 * residual decides, and a drifted residual (or a zero rh^H v, rho or omega)
 * restarts the iteration from the true residual.  opts: max_it caps the
 * iterations, max_cycles the starts (0 = no cap), rtol, pc, vbar,
 * time_slabs; restart and inner_rtol are ignored.  b, x as for
 * dirac_st_gmres (x: initial guess on entry).  stats->cycles counts the
 * starts, stats->history receives ||r|| / ||b|| per iteration.  Returns
 * DIRAC_ST_OK, DIRAC_ST_NOT_CONVERGED, DIRAC_ST_EBREAKDOWN (NaN/Inf, or a
 * restart that breaks down again before one iteration completes),
 * DIRAC_ST_ENOSPACE or DIRAC_ST_EINVAL. */
int dirac_st_bicgstab(const dirac_st_bsr *A, const void *b, void *x, const dirac_st_opts *opts,
                      void *work, size_t work_bytes, dirac_st_stats *stats, void *stream);

/* Per-time-slice diagnostics of a solution (trapezoid sums on the periodic
 * uniform mesh: nodal sums times the cell volume), for tau = 0..n_t (tau = 0
 * is psi0): out[tau][0] = int |psi|^2 (the charge monitored in Sec. 4.1),
 * out[tau][1] = the same over x_1 > x_split (the transmitted part of
 * Sec. 4.3, eq. (klein:coeffs); R's numerator is column 0 minus column 1),
 * out[tau][2 + a] = int x_{a+1} |psi|^2 with node coordinates i h (the
 * numerator of <x(t)> of Sec. 4.2).  psi0: device [S][nc] complex128;
 * x: device [nrows][nc] complex128 (a solution); out: device, (n_t + 1) x
 * (2 + d) doubles, row-major.  Deterministic (fixed summation order).
 * Enqueues on `stream`. */
int dirac_st_slice_moments(const dirac_st_problem *p, const void *psi0, const void *x, double x_split,
                           double *out, void *stream);

/* Host.  Generalised eigen-decomposition of the Galerkin time pencil used by
 * DIRAC_ST_PC_LINE: the n_t x n_t factors of the t = 1..n_t rows and columns
 * (Sec. 2.1 weak form with the t = 0 node moved to the right-hand side; App. A
 * 1D element matrices) M (mass: 2h/3, h/3 in the last row, h/6 off the
 * diagonal) and D (derivative: +-1/2 off the diagonal, 1/2 in the last
 * diagonal entry), D W = M W diag(lam), Q = W^{-1} M^{-1}.  lam: [nt], W and Q:
 * [nt][nt] row-major; complex128 interleaved, host memory.  ht: time step.
 * Fails (DIRAC_ST_EINVAL with a message) if nt is out of 1..2048 or the
 * decomposition does not pass its own residual and reconstruction checks. */
int dirac_st_time_eigen(int32_t nt, double ht, double *lam, double *W, double *Q);

/* ------------------------------------------------------------------ timing
 * Measurement support: HIP events recorded on the launch stream around the
 * launches of selected kernels, so that a caller can read the average
 * duration of a kernel while it runs inside the solver. */
enum {
  DIRAC_ST_TIMED_SPMV64 = 0,   /* y = A x, complex128 (dirac_st_spmv and inside GMRES) */
  DIRAC_ST_TIMED_SPMV32 = 1,   /* y = A x, complex64 */
  DIRAC_ST_TIMED_RESID64 = 2,  /* r = b - A x, complex128 (the FP64 true residual) */
  DIRAC_ST_TIMED_ASSEMBLE = 3, /* the block-CSR assembly kernel */
  DIRAC_ST_TIMED_SPMV_MF = 4,  /* the matrix-free operator, any precision or form */
  DIRAC_ST_TIMED_COUNT = 5
};

/* Host.  on = 1 starts recording (earlier records are dropped), on = 0 stops.
 * Process-wide; recording adds two event records per timed launch. */
int dirac_st_timing(int32_t on);

/* Host.  Number of recorded launches of `kind` and their summed duration in
 * milliseconds (waits for the recorded events). */
int dirac_st_timing_read(int32_t kind, int64_t *count, double *total_ms);

/* ------------------------------------------------------------------ batches
 * Many independent systems (Alg. 1 run for several initial fields, meshes or
 * potentials) solved together: every phase of an Arnoldi step is one launch
 * for the whole batch, its workgroups spread over the systems' tiles.
 * All systems of a batch must have the same block size nc; a batched solve
 * also needs the same dimension d for every system. */

/* Maximum number of systems in one batched call. */
#define DIRAC_ST_MAX_BATCH 1024

/* Host.  Workspace bytes of dirac_st_fgmres_batched for these systems and
 * options (0 on invalid input, see dirac_st_last_error).  A: host array of
 * nsys host pointers to assembled operators. */
size_t dirac_st_batched_workspace_bytes(int32_t nsys, const dirac_st_bsr *const *A,
                                        const dirac_st_opts *opts);

/* Flexible GMRES(m) (Sec. 2.2; Alg. 1 step 6), the same Arnoldi process as
 * dirac_st_gmres (two classical Gram-Schmidt passes, complex Givens
 * rotations, FP64 true residual at every restart, inner cycles in complex64
 * when opts->precision == 32 and x += Z y in FP64), run in lockstep over nsys
 * systems A[i] x[i] = b[i].  A system leaves the current cycle when its
 * residual estimate meets rtol (or inner_rtol for precision 32) or on a happy
 * breakdown, and retires when its FP64 residual meets rtol, or when it reaches
 * max_it / max_cycles; the others go on.  The base preconditioner opts->pc is
 * set up per system; for DIRAC_ST_PC_SPECTRAL a negative opts->vbar means
 * "half of that system's v0".  The SpMV lanes per block row are chosen by an
 * autotuner: the first call for a (nc, precision, batch size class) times each
 * candidate on the batch and caches the fastest for the process (see
 * dirac_st_batched_set_lanes).
 * A, b, x: host arrays of nsys pointers (b[i], x[i] device complex128
 * [nrows_i][nc]; x[i] is the initial guess on entry).  stats: host array of
 * nsys entries (history is not recorded; ms is the time of the whole batch).
 * work: device, 256-byte aligned, dirac_st_batched_workspace_bytes bytes.
 * Returns DIRAC_ST_OK when every system converged, DIRAC_ST_NOT_CONVERGED when
 * some did not (statistics tell which), DIRAC_ST_EBREAKDOWN if NaN/Inf appeared
 * in some system (the others are still solved), or an argument error. */
int dirac_st_fgmres_batched(int32_t nsys, const dirac_st_bsr *const *A, const void *const *b,
                            void *const *x, const dirac_st_opts *opts, void *work, size_t work_bytes,
                            dirac_st_stats *stats, void *stream);

/* Host.  Workspace bytes of dirac_st_spmv_batched for these systems (0 on
 * invalid input). */
size_t dirac_st_spmv_batched_workspace_bytes(int32_t nsys, const dirac_st_bsr *const *A);

/* y[i] = A[i] x[i] for every system in one launch (Sec. 2.2 product; like
 * dirac_st_spmv, 2x2-block operators are addressed through their stencil and
 * must come from dirac_st_assemble).  A, x, y:
 * host arrays of nsys pointers; x[i], y[i] device vectors of complex128
 * (prec 64, val64) or complex64 (prec 32, val32).  lanes: lanes per block row,
 * 4, 8, 16 or 32 for nc = 2, or 1 for the kernel that stages x in LDS per
 * tile of 32 consecutive rows of one line of axis 1 (16 lanes per complex128
 * row serving two rows, 8 per complex64 row); 64 (or 32 at prec 32) for
 * nc = 4.  Enqueues only (the small descriptor copy is synchronous). */
int dirac_st_spmv_batched(int32_t nsys, const dirac_st_bsr *const *A, int32_t prec, const void *const *x,
                          void *const *y, int32_t lanes, void *work, size_t work_bytes, void *stream);

/* Host.  Force the lanes per block row of the batched solver's SpMV for
 * (nc, prec); 0 returns to autotuning.  Process-wide. */
int dirac_st_batched_set_lanes(int32_t nc, int32_t prec, int32_t lanes);

/* Host.  Lanes the batched solver uses for a batch of `rows` block rows in total
 * (forced value, else the autotuned one; 0 if not tuned yet). */
int32_t dirac_st_batched_lanes(int32_t nc, int32_t prec, int64_t rows);

#ifdef __cplusplus
}
#endif
#endif /* DIRAC_ST_H */
