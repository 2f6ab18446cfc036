// bicgstab.hip -- BiCGSTAB with right preconditioning in complex128, the
// second Krylov solver of the paper's parallel runs (Sec. 4.4, Tables 1-3;
// algorithm of van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992)).
//
// Per iteration (r the residual of the original system, rh the shadow
// residual fixed at a (re)start):
//   p = r + beta (p - omega v);  ph = M^{-1} p;  v = A ph
//   alpha = rho / (rh^H v);      s = r - alpha v
//   sh = M^{-1} s;  t = A sh;    omega = (t^H s) / (t^H t)   (0 if t = 0)
//   x += alpha ph + omega sh;    r = s - omega t
//   rho' = rh^H r;  beta' = (rho' / rho) (alpha / omega)
// The scalars live on the device: each reduction is summed in FP64 in a fixed
// order by one workgroup, which also updates the scalars, so the iteration
// runs without host round trips; the host reads 16 bytes per iteration
// (||r||^2 and a flag) to decide when to stop.  When ||r|| meets the
// tolerance the true residual b - A x decides; if it has drifted above the
// tolerance, or rh^H v, rho or omega came out zero, the iteration restarts
// from the true residual with rh = r.  A restart that is hit again before
// any iteration completes ends the solve as a breakdown.
#include <chrono>
#include <cstring>
#include <cmath>

#include "common.hpp"
#include "krylov.hpp"
#include "readback.hpp"
#include "precond.hpp"
#include "mfspmv.hpp"
#include "spmv.hpp"

namespace dst {

struct BCtrl {
  double2 rho, alpha, omega, beta;
  double2 red[2];  // outputs of the last reduction
  // read back by the host after every iteration
  double est2;     // ||r||^2 after the update
  double flag;     // 0; 1: rh^H v = 0; 2: rho = 0; 3: omega = 0
};

__device__ inline double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return mk<double2>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// block partial of up to two sums into partial[k * nblk + blockIdx.x]
template <int K>
__device__ __forceinline__ void block_partials(double2 (&acc)[K], double2 *__restrict__ partial, int64_t nblk) {
  __shared__ double sx[K][4], sy[K][4];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const double ax = wave_sum(acc[k].x), ay = wave_sum(acc[k].y);
    if ((threadIdx.x & 63) == 0) {
      sx[k][threadIdx.x >> 6] = ax;
      sy[k][threadIdx.x >> 6] = ay;
    }
  }
  __syncthreads();
  if (threadIdx.x < K) {
    const int k = threadIdx.x;
    partial[(int64_t)k * nblk + blockIdx.x] =
        mk<double2>(sx[k][0] + sx[k][1] + sx[k][2] + sx[k][3], sy[k][0] + sy[k][1] + sy[k][2] + sy[k][3]);
  }
}

static __global__ __launch_bounds__(256) void bi_zero(double2 *__restrict__ x, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) x[e] = mk<double2>(0, 0);
}

// p = r (first) or p = r + beta (p - omega v)
__global__ __launch_bounds__(256) void bi_dir(const double2 *__restrict__ r, double2 *__restrict__ p,
                                              const double2 *__restrict__ v, const BCtrl *__restrict__ c,
                                              int first, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double2 re = r[e];
  if (first) {
    p[e] = re;
    return;
  }
  const double2 beta = c->beta, omega = c->omega;
  const double2 d = csub(p[e], cmul(omega, v[e]));
  p[e] = cadd(re, cmul(beta, d));
}

// partial[0] = sum conj(a) b;  with NORM2 also partial[1] = sum |a|^2
template <bool NORM2>
__global__ __launch_bounds__(256) void bi_dot(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                              double2 *__restrict__ partial, int64_t n, int64_t nblk) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  constexpr int K = NORM2 ? 2 : 1;
  double2 acc[K];
#pragma unroll
  for (int k = 0; k < K; k++) acc[k] = mk<double2>(0, 0);
  if (e < n) {
    const double2 av = a[e], bv = b[e];
    acc[0] = cfma_conj(acc[0], av, bv);
    if (NORM2) acc[K - 1].x = av.x * av.x + av.y * av.y;
  }
  block_partials<K>(acc, partial, nblk);
}

// s = r - alpha v
__global__ __launch_bounds__(256) void bi_s(const double2 *__restrict__ r, const double2 *__restrict__ v,
                                            double2 *__restrict__ s, const BCtrl *__restrict__ c, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  s[e] = csub(r[e], cmul(c->alpha, v[e]));
}

// x += alpha ph + omega sh;  r = s - omega t;  partials rh^H r and ||r||^2
__global__ __launch_bounds__(256) void bi_update(double2 *__restrict__ x, double2 *__restrict__ r,
                                                 const double2 *__restrict__ ph, const double2 *__restrict__ sh,
                                                 const double2 *__restrict__ s, const double2 *__restrict__ t,
                                                 const double2 *__restrict__ rh, const BCtrl *__restrict__ c,
                                                 double2 *__restrict__ partial, int64_t n, int64_t nblk) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double2 acc[2] = {mk<double2>(0, 0), mk<double2>(0, 0)};
  if (e < n) {
    const double2 alpha = c->alpha, omega = c->omega;
    x[e] = cadd(x[e], cadd(cmul(alpha, ph[e]), cmul(omega, sh[e])));
    const double2 rn = csub(s[e], cmul(omega, t[e]));
    r[e] = rn;
    acc[0] = cfma_conj(acc[0], rh[e], rn);
    acc[1].x = rn.x * rn.x + rn.y * rn.y;
  }
  block_partials<2>(acc, partial, nblk);
}

// Sums the K partial rows (fixed order, FP64) into c->red, then updates the
// scalars: stage 0 alpha, 1 omega, 2 rho / beta / est2, 3 restart (rho = ||r||^2).
template <int K>
__global__ __launch_bounds__(256) void bi_reduce(const double2 *__restrict__ partial, int64_t nblk,
                                                 BCtrl *__restrict__ c, int stage) {
  __shared__ double sx[4], sy[4];
  for (int k = 0; k < K; k++) {
    double ax = 0.0, ay = 0.0;
    const double2 *p = partial + (int64_t)k * nblk;
    int64_t b = threadIdx.x;
    // eight loads in flight per thread, summed in index order
    for (; b + 7 * 256 < nblk; b += 8 * 256) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; u++) v[u] = p[b + u * 256];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        ax += v[u].x;
        ay += v[u].y;
      }
    }
    for (; b < nblk; b += 256) {
      const double2 v = p[b];
      ax += v.x;
      ay += v.y;
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    if ((threadIdx.x & 63) == 0) {
      sx[threadIdx.x >> 6] = ax;
      sy[threadIdx.x >> 6] = ay;
    }
    __syncthreads();
    if (threadIdx.x == 0) c->red[k] = mk<double2>(sx[0] + sx[1] + sx[2] + sx[3], sy[0] + sy[1] + sy[2] + sy[3]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double2 zero = mk<double2>(0, 0);
  if (stage == 0) {
    const double2 rv = c->red[0];
    if (rv.x == 0.0 && rv.y == 0.0) {
      c->alpha = zero;
      c->flag = 1.0;
    } else {
      c->alpha = cdiv(c->rho, rv);
    }
  } else if (stage == 1) {
    const double tt = c->red[1].x;
    if (c->flag != 0.0 || !(tt > 0.0)) {
      c->omega = zero;
      if (c->flag == 0.0) c->flag = 3.0;
    } else {
      c->omega = mk<double2>(c->red[0].x / tt, c->red[0].y / tt);
    }
  } else if (stage == 2) {
    const double2 rho_new = c->red[0];
    c->est2 = c->red[1].x;
    if (c->flag == 0.0) {
      if (rho_new.x == 0.0 && rho_new.y == 0.0) {
        c->flag = 2.0;
      } else {
        c->beta = cmul(cdiv(rho_new, c->rho), cdiv(c->alpha, c->omega));
      }
    }
    c->rho = rho_new;
  } else {
    c->rho = mk<double2>(c->red[0].x, 0.0);
    c->alpha = c->omega = mk<double2>(1.0, 0.0);
    c->beta = zero;
    c->est2 = c->red[0].x;
    c->flag = 0.0;
  }
}

struct BiLayout {
  size_t r, rh, p, v, ph, s, sh, t, partial, ctrl, spec, total;
};

static BiLayout bi_layout(const dirac_st_bsr *A, const dirac_st_opts *o) {
  BiLayout L{};
  const int64_t N = A->nrows * A->nc;
  // consecutive vectors skewed by 4 KB: a power-of-two stride between the
  // streams that a pass reads together measured 5-10 % slower
  const size_t vb = align256((size_t)N * 16) + kVecSkew;
  size_t off = 0;
  size_t *vecs[] = {&L.r, &L.rh, &L.p, &L.v, &L.ph, &L.s, &L.sh, &L.t};
  for (size_t *q : vecs) {
    *q = off;
    off += vb;
  }
  L.partial = off;
  off += align256((size_t)2 * nblocks(N) * sizeof(double2));
  L.ctrl = off;
  off += align256(sizeof(BCtrl));
  L.spec = off;
  if (o->pc == DIRAC_ST_PC_SPECTRAL) off += spec_layout(&A->prob, 64).total;
  if (line_kind(o->pc)) {
    const int sl = pc_slabs(o);
    off += line_layout(&A->prob, 64, sl >= 1 && A->prob.n[0] % sl == 0 ? sl : 1).total;
  }
  L.total = off;
  return L;
}

struct BiReadback {
  double est2, flag;
};

static int bicgstab_impl(const dirac_st_bsr *A, const double2 *b, double2 *x, const dirac_st_opts *o,
                         unsigned char *work, dirac_st_stats *st, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t N = A->nrows * A->nc;
  const int64_t nblk = nblocks(N);
  const unsigned g = nblocks(N);
  const BiLayout L = bi_layout(A, o);
  double2 *r = (double2 *)(work + L.r), *rh = (double2 *)(work + L.rh), *p = (double2 *)(work + L.p);
  double2 *v = (double2 *)(work + L.v), *sv = (double2 *)(work + L.s), *t = (double2 *)(work + L.t);
  const bool pcon = o->pc != DIRAC_ST_PC_NONE;
  const bool mf = o->matrix_free != 0;
  double2 *ph = pcon ? (double2 *)(work + L.ph) : p;
  double2 *sh = pcon ? (double2 *)(work + L.sh) : sv;
  double2 *partial = (double2 *)(work + L.partial);
  BCtrl *c = (BCtrl *)(work + L.ctrl);

  Precond P;
  if (int rc = pc_setup<double>(P, A, o->pc, o->vbar, work + L.spec, s, pc_slabs(o))) return rc;

  dirac_st_stats local{};
  dirac_st_stats &S = st ? *st : local;
  double *hist = st ? st->history : nullptr;
  const int hist_len = st ? st->history_len : 0;
  S.iters = S.cycles = S.converged = 0;
  S.singular_blocks = A->singular_blocks;
  S.relres = S.est = 0.0;
  S.fallback = 0;

  // scalar readbacks land in page-locked memory when it is available
  double local_rb[8];
  double *const pinned = (double *)readback_buffer(sizeof(local_rb));
  double *const hrb = pinned ? pinned : local_rb;
  auto norm2 = [&](const double2 *a, double &out) -> int {
    bi_dot<true><<<g, 256, 0, s>>>(a, a, partial, N, nblk);
    bi_reduce<2><<<1, 256, 0, s>>>(partial, nblk, c, 3);
    DST_LAUNCHED();
    DST_HIP(hipMemcpyAsync(hrb, &c->est2, sizeof(double), hipMemcpyDeviceToHost, s));
    DST_HIP(hipStreamSynchronize(s));
    out = hrb[0];
    return 0;
  };
  double bn2 = 0.0, xn2 = 0.0;
  if (int rc = norm2(x, xn2)) return rc;
  if (int rc = norm2(b, bn2)) return rc;
  const double bnorm = sqrt(bn2);
  bool x_zero = xn2 == 0.0;
  if (!std::isfinite(bnorm)) {
    set_error("right-hand side contains NaN or Inf");
    return DIRAC_ST_EBREAKDOWN;
  }
  if (bnorm == 0.0) {
    bi_zero<<<g, 256, 0, s>>>(x, N);
    DST_LAUNCHED();
    DST_HIP(hipStreamSynchronize(s));
    S.converged = 1;
    return DIRAC_ST_OK;
  }
  int its = 0, rc_final = DIRAC_ST_NOT_CONVERGED;
  bool fresh = false;
  for (;;) {
    // (re)start from the true residual; rho = ||r||^2 with rh = r
    if (x_zero) {
      DST_HIP(hipMemcpyAsync(r, b, (size_t)N * sizeof(double2), hipMemcpyDeviceToDevice, s));
      x_zero = false;
    } else {
      DST_HIP(apply_op<double>(A, mf, A->val64, x, b, r, 1.0, true, s));
    }
    double rn2 = 0.0;
    if (int rc = norm2(r, rn2)) return rc;
    const double rn = sqrt(rn2);
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
    if (its >= o->max_it || (o->max_cycles > 0 && S.cycles >= o->max_cycles)) break;
    if (fresh) {
      set_error("BiCGSTAB broke down right after a restart");
      rc_final = DIRAC_ST_EBREAKDOWN;
      break;
    }
    S.cycles++;
    fresh = true;
    DST_HIP(hipMemcpyAsync(rh, r, (size_t)N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    bool first = true, broke = false;
    while (its < o->max_it) {
      bi_dir<<<g, 256, 0, s>>>(r, p, v, c, first ? 1 : 0, N);
      DST_LAUNCHED();
      first = false;
      if (pcon)
        if (int rc = pc_apply_base<double>(P, p, ph, 1.0, N, s)) return rc;
      DST_HIP(apply_op<double>(A, mf, A->val64, ph, nullptr, v, 1.0, false, s));
      bi_dot<false><<<g, 256, 0, s>>>(rh, v, partial, N, nblk);
      bi_reduce<1><<<1, 256, 0, s>>>(partial, nblk, c, 0);
      bi_s<<<g, 256, 0, s>>>(r, v, sv, c, N);
      DST_LAUNCHED();
      if (pcon)
        if (int rc = pc_apply_base<double>(P, sv, sh, 1.0, N, s)) return rc;
      DST_HIP(apply_op<double>(A, mf, A->val64, sh, nullptr, t, 1.0, false, s));
      bi_dot<true><<<g, 256, 0, s>>>(t, sv, partial, N, nblk);
      bi_reduce<2><<<1, 256, 0, s>>>(partial, nblk, c, 1);
      bi_update<<<g, 256, 0, s>>>(x, r, ph, sh, sv, t, rh, c, partial, N, nblk);
      bi_reduce<2><<<1, 256, 0, s>>>(partial, nblk, c, 2);
      DST_LAUNCHED();
      BiReadback rb{};
      static_assert(sizeof(rb) <= sizeof(local_rb), "fits the readback buffer");
      DST_HIP(hipMemcpyAsync(hrb, &c->est2, sizeof(rb), hipMemcpyDeviceToHost, s));
      DST_HIP(hipStreamSynchronize(s));
      memcpy(&rb, hrb, sizeof(rb));
      // rh^H v = 0: alpha and omega were set to zero, x and r are unchanged;
      // restart without counting a step
      if (rb.flag == 1.0) break;
      its++;
      fresh = false;
      const double est = sqrt(rb.est2) / bnorm;
      S.est = est;
      if (hist && its <= hist_len) hist[its - 1] = est;
      if (!std::isfinite(est)) {
        broke = true;
        break;
      }
      if (est <= o->rtol || rb.flag != 0.0) break;
    }
    if (broke) {
      set_error("NaN or Inf in BiCGSTAB");
      rc_final = DIRAC_ST_EBREAKDOWN;
      break;
    }
  }
  S.iters = its;
  DST_HIP(hipStreamSynchronize(s));
  S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return rc_final;
}

}  // namespace dst

using namespace dst;

extern "C" size_t dirac_st_bicgstab_workspace_bytes(const dirac_st_bsr *A, const dirac_st_opts *opts) {
  if (!A || !opts || (A->nc != 2 && A->nc != 4)) return 0;
  return bi_layout(A, opts).total;
}

extern "C" int dirac_st_bicgstab(const dirac_st_bsr *A, const void *b, void *x, const dirac_st_opts *opts,
                                 void *work, size_t work_bytes, dirac_st_stats *stats, void *stream) {
  clear_error();
  DST_CHECK(A != nullptr, "matrix is NULL");
  DST_CHECK(opts != nullptr, "opts is NULL");
  if (opts->matrix_free) {
    if (int rc = validate_problem(&A->prob)) return rc;
    int64_t rows = A->prob.n[0];
    for (int a = 1; a <= A->prob.d; a++) rows *= A->prob.n[a];
    DST_CHECK(A->nc == A->prob.nc && A->nrows == rows, "A->nc / A->nrows must match A->prob");
  } else {
    DST_CHECK(A->row_ptr && A->col_idx && A->val64, "matrix arrays are NULL");
    DST_CHECK(A->nc == 2 || A->nc == 4, "matrix nc must be 2 or 4 (was it assembled?)");
    DST_CHECK(A->nrows > 0 && A->nnzb > 0, "empty matrix");
  }
  DST_CHECK(b && x && work, "b, x and work must be set");
  DST_CHECK(opts->precision == 64, "BiCGSTAB runs in complex128 (precision 64)");
  if (int rc = check_pc_opts(A, opts)) return rc;
  DST_CHECK(opts->rtol > 0.0, "rtol must be positive");
  DST_CHECK(opts->max_it >= 0, "max_it must be >= 0");
  const size_t need = bi_layout(A, opts).total;
  if (work_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", work_bytes, need);
    return DIRAC_ST_ENOSPACE;
  }
  DST_CHECK(((uintptr_t)work & 255) == 0, "workspace must be 256-byte aligned");
  return bicgstab_impl(A, (const double2 *)b, (double2 *)x, opts, (unsigned char *)work, stats,
                       (hipStream_t)stream);
}
