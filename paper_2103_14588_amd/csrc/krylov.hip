// krylov.hip -- restarted GMRES(m) with right preconditioning (Sec. 2.2 and
// Alg. 1 step 6 of the paper), in complex128, or with complex64 inner cycles
// inside an FP64 refinement loop; plus the SpMV and preconditioner entry
// points of the C ABI.
//
// One cycle: r = b - A x in FP64 (val64); v_0 = r/||r||; for j = 0..m-1:
// z = M^{-1} v_j, w = A z, two classical Gram-Schmidt passes against
// v_0..v_j (the second pass re-orthogonalises), ||w||, a complex Givens
// rotation on the new Hessenberg column; the cycle ends when the rotated
// residual estimate meets the tolerance.  Then y solves the triangular
// least-squares system and x += M^{-1} (V y).
//
// Device/host split: every vector operation is a kernel on `stream`; the
// small FP64 state (Hessenberg column, rotations, g) stays on the device; the
// host reads 32 bytes back after each Arnoldi step (residual estimate, happy
// breakdown and NaN flags, next basis scale) to decide when to stop.
// Basis vectors are stored unnormalised with a scale sigma_k kept in FP64,
// so no separate normalisation pass is needed.
#include <chrono>
#include <cstddef>
#include <cstring>

#include "common.hpp"
#include "krylov.hpp"
#include "nn_host.hpp"
#include "readback.hpp"
#include "precond.hpp"
#include "spectral.hpp"
#include "mfspmv.hpp"
#include "spmv.hpp"

namespace dst {

// Norm passes: block b covers [256 kNormEpt b, 256 kNormEpt (b + 1)); each
// thread sums its kNormEpt elements in order, then the wavefront and the
// block add theirs.  One element per thread moved too few bytes per
// workgroup to keep the memory system busy.
constexpr int kNormEpt = 4;
static inline unsigned norm_blocks(int64_t n) { return (unsigned)((n + 256 * kNormEpt - 1) / (256 * kNormEpt)); }

// partial[0][b] = sum over the block's elements of |w[e]|^2
template <typename T>
__global__ __launch_bounds__(256) void norm_pass(const cx<T> *__restrict__ w,
                                                  double2 *__restrict__ partial, int64_t n) {
  __shared__ double red[4];
  cx<T> v[kNormEpt];
#pragma unroll
  for (int i = 0; i < kNormEpt; i++) {
    const int64_t e = ((int64_t)blockIdx.x * kNormEpt + i) * 256 + threadIdx.x;
    v[i] = e < n ? w[e] : mk<cx<T>>(0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kNormEpt; i++) s += (double)v[i].x * v[i].x + (double)v[i].y * v[i].y;
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[blockIdx.x] = mk<double2>(red[0] + red[1] + red[2] + red[3], 0.0);
}

// ||x||^2 and ||b||^2 in one pass: partial[b] = (block sum |x|^2, block sum |b|^2),
// each component summed exactly as norm_pass sums it
__global__ __launch_bounds__(256) void norm_pass2(const double2 *__restrict__ x, const double2 *__restrict__ b,
                                                  double2 *__restrict__ partial, int64_t n) {
  __shared__ double red[2][4];
  double2 vx[kNormEpt], vb[kNormEpt];
#pragma unroll
  for (int i = 0; i < kNormEpt; i++) {
    const int64_t e = ((int64_t)blockIdx.x * kNormEpt + i) * 256 + threadIdx.x;
    vx[i] = e < n ? x[e] : mk<double2>(0, 0);
    vb[i] = e < n ? b[e] : mk<double2>(0, 0);
  }
  double sx = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < kNormEpt; i++) {
    sx += vx[i].x * vx[i].x + vx[i].y * vx[i].y;
    sb += vb[i].x * vb[i].x + vb[i].y * vb[i].y;
  }
  sx = wave_sum(sx);
  sb = wave_sum(sb);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sx;
    red[1][threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    partial[blockIdx.x] = mk<double2>(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                                      red[1][0] + red[1][1] + red[1][2] + red[1][3]);
}

__global__ __launch_bounds__(256) void zero_c128(double2 *x, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) x[e] = mk<double2>(0, 0);
}

static int maxk_bucket(int jp1) {
  return jp1 <= 1 ? 1 : jp1 <= 2 ? 2 : jp1 <= 4 ? 4 : jp1 <= 8 ? 8 : jp1 <= 16 ? 16 : jp1 <= 32 ? 32 : 64;
}

// Passes over at most four basis vectors move too few bytes per thread to
// keep the memory system busy with one element each: their threads take four.
constexpr int kSmallSetEpt = 4;
static int64_t pass_blocks(int64_t n, int mk) {
  const int64_t per = 256 * (mk <= 4 ? kSmallSetEpt : 1);
  return (n + per - 1) / per;
}

template <typename T, int MODE>
static hipError_t launch_pass_mk(int mk, const cx<T> *V, int64_t ldv, int jp1, cx<T> *w,
                                 const double2 *coef, double2 *partial, int64_t n, hipStream_t s) {
  const unsigned g = (unsigned)pass_blocks(n, mk);
  constexpr int E = kSmallSetEpt;
  switch (mk) {
    case 1: cgs_pass<T, 1, MODE, E><<<g, 256, 0, s>>>(V, ldv, jp1, w, coef, partial, n); break;
    case 2: cgs_pass<T, 2, MODE, E><<<g, 256, 0, s>>>(V, ldv, jp1, w, coef, partial, n); break;
    case 4: cgs_pass<T, 4, MODE, E><<<g, 256, 0, s>>>(V, ldv, jp1, w, coef, partial, n); break;
    case 8: cgs_pass<T, 8, MODE><<<g, 256, 0, s>>>(V, ldv, jp1, w, coef, partial, n); break;
    case 16: cgs_pass<T, 16, MODE><<<g, 256, 0, s>>>(V, ldv, jp1, w, coef, partial, n); break;
    case 32: cgs_pass<T, 32, MODE><<<g, 256, 0, s>>>(V, ldv, jp1, w, coef, partial, n); break;
    default: cgs_pass<T, 64, MODE><<<g, 256, 0, s>>>(V, ldv, jp1, w, coef, partial, n); break;
  }
  return hipGetLastError();
}

// the fused update + dots pass handles every Gram-Schmidt set size (the
// basis entries are re-read for the dots, not held in registers)
template <typename T>
static bool fused_updots_ok(int) {
  return true;
}

template <typename T>
static hipError_t launch_updots(int mk, const cx<T> *V, int64_t ldv, int jp1, cx<T> *w,
                                const double2 *coef, double2 *partial, int64_t n, hipStream_t s) {
  return launch_pass_mk<T, UPDOTS>(mk, V, ldv, jp1, w, coef, partial, n, s);
}

// ------------------------------------------------------------ layout
struct GmresLayout {
  size_t V, z, u, r64, partial, ctrl, spec, Z, nn, total;
  int64_t ldv;  // elements between basis vectors
};

static GmresLayout gmres_layout(const dirac_st_bsr *A, const dirac_st_opts *o, bool flexible) {
  GmresLayout L{};
  const int64_t N = A->nrows * A->nc;
  const size_t cs = o->precision == 32 ? 8 : 16;
  // consecutive vectors skewed by 4 KB: a power-of-two stride between the
  // streams that a pass reads together measured 5-10 % slower
  const size_t vb = align256((size_t)N * cs) + kVecSkew;
  L.ldv = (int64_t)(vb / cs);
  size_t off = 0;
  L.V = off;
  off += vb * (size_t)(o->restart + 1);
  L.z = off;
  off += vb;
  L.u = off;
  off += vb;
  L.r64 = off;
  if (o->precision == 32) off += align256((size_t)N * 16);
  L.partial = off;
  off += align256((size_t)nblocks(N) * kMaxRestart * sizeof(double2));
  L.ctrl = off;
  off += align256(sizeof(Ctrl));
  L.spec = off;
  if (o->pc == DIRAC_ST_PC_SPECTRAL) off += spec_layout(&A->prob, o->precision).total;
  if (line_kind(o->pc)) {
    // an invalid slab count is rejected by the solver; size as one slab (the largest)
    const int sl = pc_slabs(o);
    off += line_layout(&A->prob, o->precision, sl >= 1 && A->prob.n[0] % sl == 0 ? sl : 1).total;
  }
  L.Z = off;
  if (flexible) off += vb * (size_t)o->restart;
  L.nn = off;
  if (flexible && A->prob.d == 2)
    off += nn_layout(A->prob.n[0], A->prob.n[2], A->prob.n[1], false).total;
  L.total = off;
  return L;
}

// Full preconditioner on the true vector scale * v (unit norm in GMRES):
// base part plus, when the network is on, (1/sqrt(n)) N(sqrt(n) scale v).
template <typename T>
static int pc_apply(const Precond &P, const cx<T> *v, cx<T> *z, double scale, int64_t N,
                    hipStream_t s) {
  const bool base = P.kind != DIRAC_ST_PC_NONE;
  if (base)
    if (int rc = pc_apply_base<T>(P, v, z, scale, N, s)) return rc;
  if (P.nn_on) {
    const dirac_st_problem &p = P.A->prob;
    const double rn = sqrt((double)N);
    return nn_apply_add(P.nn, p.n[0], p.n[2], p.n[1], v, sizeof(T) == 8 ? 64 : 32, rn * scale,
                        (P.nn->out_gain != 0.f ? (double)P.nn->out_gain : 1.0) / rn, z, base ? 1 : 0,
                        P.nnwork, s);
  }
  if (!base) {
    set_error("no preconditioner to apply");
    return DIRAC_ST_EINVAL;
  }
  return 0;
}

// ------------------------------------------------------------ GMRES
struct Readback {
  double est_abs, happy, finite, sigma_next;
};
static_assert(sizeof(Readback) <= 8 * sizeof(double), "fits the solver's readback buffers");

template <typename T>
static int gmres_impl(const dirac_st_bsr *A, const double2 *b, double2 *x, const dirac_st_opts *o,
                      unsigned char *work, dirac_st_stats *st, hipStream_t s, bool flexible,
                      const dirac_st_nn *net) {
  using C = cx<T>;
  const auto t_start = std::chrono::steady_clock::now();
  const int nc = A->nc;
  const int64_t N = A->nrows * nc;
  const int m = o->restart;
  const GmresLayout L = gmres_layout(A, o, flexible);
  C *V = (C *)(work + L.V);
  C *z = (C *)(work + L.z);
  C *u = (C *)(work + L.u);
  double2 *r64 = (double2 *)(work + L.r64);
  double2 *partial = (double2 *)(work + L.partial);
  Ctrl *ctrl = (Ctrl *)(work + L.ctrl);
  C *Zb = (C *)(work + L.Z);
  const void *val = sizeof(T) == 8 ? A->val64 : A->val32;
  const bool mf = o->matrix_free != 0;

  Precond P;
  if (int rc = pc_setup<T>(P, A, o->pc, o->vbar, work + L.spec, s, pc_slabs(o))) return rc;
  if (net) {
    P.nn = net;
    P.nn_on = true;
    P.nnwork = work + L.nn;
  }
  zero_ctrl<<<8, 256, 0, s>>>(ctrl);
  DST_LAUNCHED();

  // scalar readbacks land in page-locked memory when it is available
  double local_rb[8];
  double *const pinned = (double *)readback_buffer(sizeof(local_rb));
  double *const hrb = pinned ? pinned : local_rb;
  auto read_norm = [&](const double2 *v, double &out) -> int {
    norm_pass<double><<<norm_blocks(N), 256, 0, s>>>(v, partial, N);
    reduce_partials<<<1, 256, 0, s>>>(partial, norm_blocks(N), ctrl, 1, 0);
    DST_LAUNCHED();
    DST_HIP(hipMemcpyAsync(hrb, &ctrl->dots_norm2, sizeof(double), hipMemcpyDeviceToHost, s));
    DST_HIP(hipStreamSynchronize(s));
    out = sqrt(hrb[0]);
    return 0;
  };

  dirac_st_stats local{};
  dirac_st_stats &S = st ? *st : local;
  double *hist = st ? st->history : nullptr;
  const int hist_len = st ? st->history_len : 0;
  S.iters = S.cycles = S.converged = 0;
  S.singular_blocks = A->singular_blocks;
  S.relres = S.est = 0.0;
  S.fallback = 0;
  double relres_prev = -1.0;

  // a zero initial guess needs no first SpMV: its residual is b.  ||x||^2 and
  // ||b||^2 come back in one copy (the estimate slot and the norm^2 slot,
  // which the control block keeps two doubles apart)
  double xnorm = 0.0, bnorm = 0.0;
  double2 *rbuf = sizeof(T) == 8 ? (double2 *)V : r64;
  {
    norm_pass2<<<norm_blocks(N), 256, 0, s>>>(x, b, partial, N);
    reduce_partials<<<1, 256, 0, s>>>(partial, norm_blocks(N), ctrl, 2, 0);
    DST_LAUNCHED();
    // the residual of a zero initial guess is b: the copy is queued before the
    // norms are read back, so it runs while the host waits (with a nonzero x
    // the first residual product overwrites it)
    DST_HIP(hipMemcpyAsync(rbuf, b, (size_t)N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    static_assert(offsetof(Ctrl, est_abs) == offsetof(Ctrl, dots_norm2) + 2 * sizeof(double),
                  "norm^2 and estimate slots");
    DST_HIP(hipMemcpyAsync(hrb, &ctrl->dots_norm2, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    DST_HIP(hipStreamSynchronize(s));
    xnorm = sqrt(hrb[2]);
    bnorm = sqrt(hrb[0]);
  }
  bool x_zero = xnorm == 0.0;
  if (!std::isfinite(bnorm)) {
    set_error("right-hand side contains NaN or Inf");
    return DIRAC_ST_EBREAKDOWN;
  }
  if (bnorm == 0.0) {
    zero_c128<<<nblocks(N), 256, 0, s>>>(x, N);
    DST_LAUNCHED();
    DST_HIP(hipStreamSynchronize(s));
    S.converged = 1;
    return DIRAC_ST_OK;
  }
  int its = 0, rc_final = DIRAC_ST_NOT_CONVERGED;
  for (;;) {
    // true residual in FP64
    double rn = 0.0;
    if (x_zero) {
      rn = bnorm;  // rbuf already holds b
      x_zero = false;
    } else {
      DST_HIP(apply_op<double>(A, mf, A->val64, x, b, rbuf, 1.0, true, s));
      if (int rc = read_norm(rbuf, rn)) return rc;
    }
    S.relres = rn / bnorm;
    if (!std::isfinite(rn)) {
      set_error("NaN or Inf in the residual");
      rc_final = DIRAC_ST_EBREAKDOWN;
      break;
    }
    if (S.relres <= o->rtol) {
      S.converged = 1;
      rc_final = DIRAC_ST_OK;
      break;
    }
    // network fallback: a cycle that cut the residual by less than 1%
    if (P.nn_on && relres_prev > 0.0 && S.relres > 0.99 * relres_prev) {
      P.nn_on = false;
      S.fallback = 1;
    }
    relres_prev = S.relres;
    if (its >= o->max_it || (o->max_cycles > 0 && S.cycles >= o->max_cycles)) break;
    S.cycles++;
    if (sizeof(T) == 8) {
      cycle_init<<<1, 64, 0, s>>>(ctrl, rn, 1.0 / rn);
    } else {
      scale_convert<T><<<nblocks(N), 256, 0, s>>>(r64, 1.0 / rn, V, N);
      cycle_init<<<1, 64, 0, s>>>(ctrl, rn, 1.0);
    }
    DST_LAUNCHED();
    double sigma_j = sizeof(T) == 8 ? 1.0 / rn : 1.0;
    int k = 0;
    bool broke = false;
    for (int j = 0; j < m && its < o->max_it; j++) {
      C *vj = V + (int64_t)j * L.ldv;
      C *w = V + (int64_t)(j + 1) * L.ldv;
      // w = A M^{-1} v_j
      if (P.kind == DIRAC_ST_PC_NONE && !P.nn_on && !flexible) {
        DST_HIP(apply_op<T>(A, mf, val, vj, nullptr, w, (T)sigma_j, false, s));
      } else if (P.kind == DIRAC_ST_PC_NONE && !P.nn_on) {
        // flexible without any preconditioner: z_j = v_j
        C *zj = Zb + (int64_t)j * L.ldv;
        scale_copy<T><<<nblocks(N), 256, 0, s>>>(vj, sigma_j, zj, N);
        DST_LAUNCHED();
        DST_HIP(apply_op<T>(A, mf, val, zj, nullptr, w, (T)1, false, s));
      } else {
        C *zj = flexible ? Zb + (int64_t)j * L.ldv : z;
        if (int rc = pc_apply<T>(P, vj, zj, sigma_j, N, s)) return rc;
        DST_HIP(apply_op<T>(A, mf, val, zj, nullptr, w, (T)1, false, s));
      }
      const int jp1 = j + 1, mk = maxk_bucket(jp1);
      const int64_t nbk = pass_blocks(N, mk);  // partial sums per coefficient
      // pass 1: h1 = V^H w
      DST_HIP((launch_pass_mk<T, DOTS>(mk, V, L.ldv, jp1, w, nullptr, partial, N, s)));
      reduce_partials<<<jp1, 256, 0, s>>>(partial, nbk, ctrl, 0, 1);
      DST_LAUNCHED();
      // pass 2: w -= V h1, h2 = V^H w
      if (fused_updots_ok<T>(mk)) {
        DST_HIP(launch_updots<T>(mk, V, L.ldv, jp1, w, ctrl->coef, partial, N, s));
      } else {
        DST_HIP((launch_pass_mk<T, UPDATE>(mk, V, L.ldv, jp1, w, ctrl->coef, partial, N, s)));
        DST_HIP((launch_pass_mk<T, DOTS>(mk, V, L.ldv, jp1, w, nullptr, partial, N, s)));
      }
      reduce_partials<<<jp1, 256, 0, s>>>(partial, nbk, ctrl, 0, 2);
      DST_LAUNCHED();
      // pass 3: w -= V h2, ||w||^2
      DST_HIP((launch_pass_mk<T, UPNORM>(mk, V, L.ldv, jp1, w, ctrl->coef, partial, N, s)));
      reduce_partials<<<1, 256, 0, s>>>(partial, nbk, ctrl, 1, 0);
      givens_step<<<1, 64, 0, s>>>(ctrl, j);
      DST_LAUNCHED();
      Readback rb{};
      DST_HIP(hipMemcpyAsync(hrb, &ctrl->est_abs, sizeof(rb), hipMemcpyDeviceToHost, s));
      DST_HIP(hipStreamSynchronize(s));
      memcpy(&rb, hrb, sizeof(rb));
      its++;
      k = j + 1;
      const double est = rb.est_abs / bnorm;
      S.est = est;
      if (hist && its <= hist_len) hist[its - 1] = est;
      if (rb.finite == 0.0 || !std::isfinite(est)) {
        broke = true;
        break;
      }
      sigma_j = rb.sigma_next;
      if (est <= o->rtol || rb.happy != 0.0) break;
      if (sizeof(T) == 4 && o->inner_rtol > 0.0 && rb.est_abs <= o->inner_rtol * rn) break;
    }
    if (broke && P.nn_on) {
      // network output not finite: drop this cycle, continue with the base
      P.nn_on = false;
      S.fallback = 1;
      relres_prev = -1.0;
      continue;
    }
    if (broke) {
      set_error("NaN or Inf in the Arnoldi process");
      rc_final = DIRAC_ST_EBREAKDOWN;
      break;
    }
    // x += M^{-1} V y  (flexible: x += Z y)
    back_substitute<<<1, 64, 0, s>>>(ctrl, k, flexible ? 1 : 0);
    DST_LAUNCHED();
    if (flexible) {
      combine<T, double, true><<<nblocks(N), 256, 0, s>>>(Zb, L.ldv, k, ctrl->coef, x, N);
      DST_LAUNCHED();
    } else if (P.kind == DIRAC_ST_PC_NONE) {
      combine<T, double, true><<<nblocks(N), 256, 0, s>>>(V, L.ldv, k, ctrl->coef, x, N);
      DST_LAUNCHED();
    } else {
      combine<T, T, false><<<nblocks(N), 256, 0, s>>>(V, L.ldv, k, ctrl->coef, u, N);
      DST_LAUNCHED();
      if (int rc = pc_apply<T>(P, u, z, 1.0, N, s)) return rc;
      add_into64<T><<<nblocks(N), 256, 0, s>>>(x, z, N);
      DST_LAUNCHED();
    }
  }
  S.iters = its;
  DST_HIP(hipStreamSynchronize(s));
  S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return rc_final;
}

static int check_bsr(const dirac_st_bsr *A) {
  DST_CHECK(A != nullptr, "matrix is NULL");
  DST_CHECK(A->row_ptr && A->col_idx && A->val64, "matrix arrays are NULL");
  DST_CHECK(A->nc == 2 || A->nc == 4, "matrix nc must be 2 or 4 (was it assembled?)");
  DST_CHECK(A->nrows > 0 && A->nnzb > 0, "empty matrix");
  return 0;
}

// solvers: with the matrix-free operator only the problem (and the row count
// it implies) must be valid
static int check_solver_matrix(const dirac_st_bsr *A, const dirac_st_opts *o) {
  DST_CHECK(A != nullptr, "matrix is NULL");
  DST_CHECK(o != nullptr, "opts is NULL");
  if (!o->matrix_free) return check_bsr(A);
  if (int rc = validate_problem(&A->prob)) return rc;
  DST_CHECK(A->nc == A->prob.nc, "A->nc must equal prob.nc");
  int64_t rows = A->prob.n[0];
  for (int a = 1; a <= A->prob.d; a++) rows *= A->prob.n[a];
  DST_CHECK(A->nrows == rows, "A->nrows must be the row count of A->prob");
  return 0;
}

}  // namespace dst

using namespace dst;

extern "C" int dirac_st_spmv(const dirac_st_bsr *A, int32_t prec, const void *x, void *y,
                             void *stream) {
  clear_error();
  if (int rc = check_bsr(A)) return rc;
  DST_CHECK(prec == 64 || prec == 32, "prec must be 64 or 32");
  DST_CHECK(x && y, "x and y must be set");
  DST_CHECK(x != y, "x and y must not overlap");
  DST_CHECK(prec == 64 || A->val32, "prec 32 needs val32");
  DST_CHECK(((uintptr_t)x & 15) == 0 && ((uintptr_t)y & 15) == 0, "x, y must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (prec == 64)
    DST_HIP(launch_spmv_st<double>(A, A->val64, x, nullptr, y, 1.0, false, s));
  else
    DST_HIP(launch_spmv_st<float>(A, A->val32, x, nullptr, y, 1.0f, false, s));
  return DIRAC_ST_OK;
}

extern "C" int dirac_st_spmv_mf(const dirac_st_problem *p, int32_t prec, const void *x, void *y, void *stream) {
  clear_error();
  DST_CHECK(p != nullptr, "problem is NULL");
  if (int rc = validate_problem(p)) return rc;
  DST_CHECK(prec == 64 || prec == 32, "prec must be 64 or 32");
  DST_CHECK(x && y, "x and y must be set");
  DST_CHECK(x != y, "x and y must not overlap");
  const size_t al = prec == 64 ? 16 : 8;
  DST_CHECK(((uintptr_t)x % al) == 0 && ((uintptr_t)y % al) == 0, "x, y must be aligned to their element size");
  hipStream_t s = (hipStream_t)stream;
  if (prec == 64)
    DST_HIP(launch_spmv_mf<double>(p, x, nullptr, y, 1.0, false, s));
  else
    DST_HIP(launch_spmv_mf<float>(p, x, nullptr, y, 1.0f, false, s));
  return DIRAC_ST_OK;
}

extern "C" int dirac_st_rhs_mf(const dirac_st_problem *p, const void *psi0, void *b, void *stream) {
  clear_error();
  DST_CHECK(p != nullptr, "problem is NULL");
  if (int rc = validate_problem(p)) return rc;
  DST_CHECK(psi0 && b, "psi0 and b must be set");
  DST_CHECK(((uintptr_t)psi0 & 15) == 0 && ((uintptr_t)b & 15) == 0, "psi0, b must be 16-byte aligned");
  DST_HIP(launch_rhs_mf(p, psi0, b, (hipStream_t)stream));
  return DIRAC_ST_OK;
}

extern "C" size_t dirac_st_workspace_bytes(const dirac_st_bsr *A, const dirac_st_opts *o,
                                           int32_t flexible) {
  if (!A || !o || (A->nc != 2 && A->nc != 4)) return 0;
  dirac_st_opts oo = *o;
  if (oo.restart < 1) oo.restart = 1;
  if (oo.restart > kMaxRestart) oo.restart = kMaxRestart;
  return gmres_layout(A, &oo, flexible != 0).total;
}

extern "C" int dirac_st_pc_apply(const dirac_st_bsr *A, const dirac_st_opts *opts, const void *v, void *z,
                                 void *work, size_t work_bytes, void *stream) {
  clear_error();
  if (int rc = check_bsr(A)) return rc;
  DST_CHECK(opts != nullptr, "opts is NULL");
  const int pc = opts->pc, prec = opts->precision;
  DST_CHECK(prec == 64 || prec == 32, "precision must be 64 or 32");
  DST_CHECK(pc != DIRAC_ST_PC_NONE, "no preconditioner to apply");
  if (int rc = check_pc_opts(A, opts)) return rc;
  DST_CHECK(v && z && v != z, "v and z must be set and distinct");
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = A->nrows * A->nc;
  if (pc == DIRAC_ST_PC_SPECTRAL || line_kind(pc)) {
    const size_t need = pc == DIRAC_ST_PC_SPECTRAL ? spec_layout(&A->prob, prec).total
                                                   : line_layout(&A->prob, prec, pc_slabs(opts)).total;
    DST_CHECK(work != nullptr, "this preconditioner needs a workspace");
    DST_CHECK(((uintptr_t)work & 255) == 0, "workspace must be 256-byte aligned");
    if (work_bytes < need) {
      set_error("workspace too small: %zu < %zu", work_bytes, need);
      return DIRAC_ST_ENOSPACE;
    }
  }
  Precond P;
  if (prec == 64) {
    if (int rc = pc_setup<double>(P, A, pc, opts->vbar, (unsigned char *)work, s, pc_slabs(opts))) return rc;
    return pc_apply<double>(P, (const double2 *)v, (double2 *)z, 1.0, N, s);
  }
  if (int rc = pc_setup<float>(P, A, pc, opts->vbar, (unsigned char *)work, s, pc_slabs(opts))) return rc;
  return pc_apply<float>(P, (const float2 *)v, (float2 *)z, 1.0, N, s);
}

extern "C" int dirac_st_gmres(const dirac_st_bsr *A, const void *b, void *x,
                              const dirac_st_opts *opts, void *work, size_t work_bytes,
                              dirac_st_stats *stats, void *stream) {
  clear_error();
  DST_CHECK(opts != nullptr, "opts is NULL");
  if (int rc = check_solver_matrix(A, opts)) return rc;
  DST_CHECK(b && x && work, "b, x and work must be set");
  DST_CHECK(opts->restart >= 1 && opts->restart <= kMaxRestart, "restart must be in 1..%d",
            kMaxRestart);
  DST_CHECK(opts->precision == 64 || opts->precision == 32, "precision must be 64 or 32");
  DST_CHECK(opts->precision == 64 || A->val32 || opts->matrix_free, "precision 32 needs val32");
  if (int rc = check_pc_opts(A, opts)) return rc;
  DST_CHECK(opts->rtol > 0.0, "rtol must be positive");
  DST_CHECK(opts->max_it >= 0, "max_it must be >= 0");
  const size_t need = gmres_layout(A, opts, false).total;
  if (work_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", work_bytes, need);
    return DIRAC_ST_ENOSPACE;
  }
  DST_CHECK(((uintptr_t)work & 255) == 0, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  // With room for the preconditioned vectors, keep them (flexible form): the
  // end-of-cycle update is then x += Z y, one preconditioner application
  // fewer per cycle, same iterates.
  const bool keep_z = opts->pc != DIRAC_ST_PC_NONE && work_bytes >= gmres_layout(A, opts, true).total;
  if (opts->precision == 64)
    return gmres_impl<double>(A, (const double2 *)b, (double2 *)x, opts, (unsigned char *)work,
                              stats, s, keep_z, nullptr);
  return gmres_impl<float>(A, (const double2 *)b, (double2 *)x, opts, (unsigned char *)work, stats,
                           s, keep_z, nullptr);
}

extern "C" int dirac_st_fgmres_nn(const dirac_st_bsr *A, const void *b, void *x,
                                  const dirac_st_nn *net, const dirac_st_opts *opts, void *work,
                                  size_t work_bytes, dirac_st_stats *stats, void *stream) {
  clear_error();
  DST_CHECK(opts != nullptr, "opts is NULL");
  if (int rc = check_solver_matrix(A, opts)) return rc;
  DST_CHECK(b && x && work, "b, x and work must be set");
  DST_CHECK(opts->restart >= 1 && opts->restart <= kMaxRestart, "restart must be in 1..%d",
            kMaxRestart);
  DST_CHECK(opts->precision == 64 || opts->precision == 32, "precision must be 64 or 32");
  DST_CHECK(opts->precision == 64 || A->val32 || opts->matrix_free, "precision 32 needs val32");
  if (int rc = check_pc_opts(A, opts)) return rc;
  DST_CHECK(opts->rtol > 0.0, "rtol must be positive");
  DST_CHECK(opts->max_it >= 0, "max_it must be >= 0");
  DST_CHECK(!net || A->prob.d == 2, "the network preconditioner is for 2+1D operators");
  DST_CHECK(!net || (net->params && net->w16 && net->wt16), "network arrays are NULL");
  const size_t need = gmres_layout(A, opts, true).total;
  if (work_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", work_bytes, need);
    return DIRAC_ST_ENOSPACE;
  }
  DST_CHECK(((uintptr_t)work & 255) == 0, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (opts->precision == 64)
    return gmres_impl<double>(A, (const double2 *)b, (double2 *)x, opts, (unsigned char *)work,
                              stats, s, true, net);
  return gmres_impl<float>(A, (const double2 *)b, (double2 *)x, opts, (unsigned char *)work, stats,
                           s, true, net);
}
