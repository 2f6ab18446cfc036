// krylov.hpp -- vector kernels of restarted GMRES: fused classical
// Gram-Schmidt passes (CGS2), partial-sum reduction, Givens rotations and
// back substitution (FP64), basis combinations and updates.
#pragma once

#include "common.hpp"

namespace dst {

constexpr int kMaxRestart = 64;

// Small FP64 state of one GMRES cycle, kept in device memory.
struct Ctrl {
  double2 h1[kMaxRestart + 1];    // first Gram-Schmidt coefficients
  double2 h2[kMaxRestart + 1];    // second (re-orthogonalisation) coefficients
  double2 coef[kMaxRestart + 1];  // coefficients used by the next update pass
  double2 H[kMaxRestart][kMaxRestart + 1];  // rotated Hessenberg, column-major H[col][row]
  double2 cs[kMaxRestart], sn[kMaxRestart];
  double2 g[kMaxRestart + 1];     // rotated right-hand side beta e_1
  double2 y[kMaxRestart];         // least-squares solution
  double sigma[kMaxRestart + 1];  // basis vector k is sigma[k] * (stored vector k)
  double dots_norm2;              // reduction output of norm passes
  double w0norm2;                 // estimate of ||A z_j||^2 before orthogonalisation
  // read back by the host after every Arnoldi step
  double est_abs;                 // |g_{j+1}|
  double happy;                   // 1 if h_{j+1,j} <= 1e-14 ||A z_j||
  double finite;                  // 0 if NaN/Inf appeared
  double sigma_next;              // scale of the new basis vector
};

// ------------------------------------------------------------ wave helpers
// Butterfly reduce-scatter across the 64 lanes of a wavefront: on entry each
// lane holds K values; on exit lane l (l < K) holds the wavefront sum of value l.
template <int K, typename S>
__device__ inline void wave_reduce_scatter(S (&v)[K][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int half = K / 2; half >= 1; half >>= 1) {
    const bool up = (lane & half) != 0;
#pragma unroll
    for (int i = 0; i < half; i++) {
#pragma unroll
      for (int c = 0; c < 2; c++) {
        S send = up ? v[i][c] : v[i + half][c];
        S keep = up ? v[i + half][c] : v[i][c];
        v[i][c] = keep + __shfl_xor(send, half, 64);
      }
    }
  }
#pragma unroll
  for (int off = K; off < 64; off <<= 1) {
    v[0][0] += __shfl_xor(v[0][0], off, 64);
    v[0][1] += __shfl_xor(v[0][1], off, 64);
  }
}

template <typename S>
__device__ inline S wave_sum(S v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------------ pass kernels
// Each thread takes EPT elements: block b covers [256 EPT b, 256 EPT (b + 1)),
// thread t the elements 256 (EPT b + i) + t, i < EPT.
// Modes:
//   DOTS    partial[k][b] = sum_e conj(V_k[e]) w[e], k < jp1   (tiles of 32)
//   UPDOTS  w[e] -= sum_k V_k[e] coef[k]; partial[k][b] = sum conj(V_k[e]) w_new[e]
//   UPNORM  w[e] -= sum_k V_k[e] coef[k]; partial[0][b] = sum |w_new[e]|^2
//   UPDATE  w[e] -= sum_k V_k[e] coef[k]
// A thread sums its own elements in order before the wavefront butterfly;
// with EPT = 1 every product enters the butterfly as it is.
enum PassMode { DOTS = 0, UPDOTS = 1, UPNORM = 2, UPDATE = 3 };

template <typename T, int MAXK, int MODE, int EPT = 1>
__device__ __forceinline__ void cgs_block(int64_t blk, int64_t nblk, const cx<T> *__restrict__ V, int64_t ldv, int jp1,
                                                 cx<T> *__restrict__ w,
                                                 const double2 *__restrict__ coef,
                                                 double2 *__restrict__ partial, int64_t n) {
  using C = cx<T>;
  constexpr int KT = MAXK < 32 ? MAXK : 32;
  __shared__ double red[4][KT][2];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t e[EPT];
  bool in[EPT];
  C we[EPT];
#pragma unroll
  for (int i = 0; i < EPT; i++) {
    e[i] = (blk * EPT + i) * 256 + threadIdx.x;
    in[i] = e[i] < n;
    we[i] = in[i] ? w[e[i]] : mk<C>(0, 0);
  }
  // partial[k][blk] = sum over the block's elements of conj(V_k) x, one
  // butterfly per tile of basis vectors
  auto dots = [&](const C(&x)[EPT]) {
#pragma unroll 1
    for (int t0 = 0; t0 < MAXK; t0 += KT) {
      if (t0 >= jp1) break;
      T p[KT][2];
#pragma unroll
      for (int q = 0; q < KT; q++) p[q][0] = p[q][1] = (T)0;
#pragma unroll
      for (int i = 0; i < EPT; i++) {
#pragma unroll
        for (int q = 0; q < KT; q++) {
          const int k = t0 + q;
          const C v = (in[i] && k < jp1) ? V[(int64_t)k * ldv + e[i]] : mk<C>(0, 0);
          const C pr = cfma_conj(mk<C>(p[q][0], p[q][1]), v, x[i]);
          p[q][0] = pr.x;
          p[q][1] = pr.y;
        }
      }
      wave_reduce_scatter<KT>(p);
      if (lane < KT) {
        red[wv][lane][0] = (double)p[0][0];
        red[wv][lane][1] = (double)p[0][1];
      }
      __syncthreads();
      if (threadIdx.x < KT && t0 + threadIdx.x < jp1) {
        const int q = threadIdx.x;
        double2 s = mk<double2>(red[0][q][0] + red[1][q][0] + red[2][q][0] + red[3][q][0],
                                red[0][q][1] + red[1][q][1] + red[2][q][1] + red[3][q][1]);
        partial[(int64_t)(t0 + q) * nblk + blk] = s;
      }
      __syncthreads();
    }
  };
  if (MODE == DOTS) {
    dots(we);
    return;
  }
  // update part (coefficients are uniform: scalar loads)
  C acc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; i++) acc[i] = we[i];
#pragma unroll
  for (int k = 0; k < MAXK; k++) {
    if (k < jp1) {
      const double2 c = coef[k];
      const C ck = mk<C>((T)c.x, (T)c.y);
#pragma unroll
      for (int i = 0; i < EPT; i++) {
        const C v = in[i] ? V[(int64_t)k * ldv + e[i]] : mk<C>(0, 0);
        acc[i] = cfms(acc[i], v, ck);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; i++)
    if (in[i]) w[e[i]] = acc[i];
  if (MODE == UPDATE) return;
  if (MODE == UPNORM) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < EPT; i++)
      s += in[i] ? (double)acc[i].x * acc[i].x + (double)acc[i].y * acc[i].y : 0.0;
    s = wave_sum(s);
    if (lane == 0) red[wv][0][0] = s;
    __syncthreads();
    if (threadIdx.x == 0)
      partial[blk] =
          mk<double2>(red[0][0][0] + red[1][0][0] + red[2][0][0] + red[3][0][0], 0.0);
    return;
  }
  // UPDOTS: products with the updated entries.  The basis entries are read a
  // second time (the wavefront's lines are still in the caches) rather than
  // held in registers: holding them halved the occupancy and cost more than
  // the second read.
  if (MODE == UPDOTS) dots(acc);
}

template <typename T, int MAXK, int MODE, int EPT = 1>
__global__ __launch_bounds__(256) void cgs_pass(const cx<T> *__restrict__ V, int64_t ldv, int jp1,
                                                 cx<T> *__restrict__ w,
                                                 const double2 *__restrict__ coef,
                                                 double2 *__restrict__ partial, int64_t n) {
  cgs_block<T, MAXK, MODE, EPT>(blockIdx.x, gridDim.x, V, ldv, jp1, w, coef, partial, n);
}

// Sum partial[k][b] over blocks b (fixed order, FP64); one workgroup per k.
// Layout: partial[k * nblk + b], contiguous per coefficient.
// what: 0 -> Gram-Schmidt coefficients into dst (h1 or h2) and coef = sigma_k h_k
//       1 -> norm^2 into ctrl->dots_norm2
//       2 -> a pair of norms^2: first into ctrl->est_abs, second into ctrl->dots_norm2
__device__ __forceinline__ void reduce_coef(int k, const double2 *__restrict__ partial, int64_t nblk,
                                   Ctrl *__restrict__ ctrl, int what, int which) {
  __shared__ double sx[4], sy[4];
  double ax = 0.0, ay = 0.0;
  const double2 *p = partial + (int64_t)k * nblk;
  int64_t b = threadIdx.x;
  // eight loads in flight per thread; each thread still sums its entries in
  // index order, so the result does not depend on the unrolling
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
  if (threadIdx.x == 0) {
    double x = sx[0] + sx[1] + sx[2] + sx[3], y = sy[0] + sy[1] + sy[2] + sy[3];
    if (what == 1) {
      ctrl->dots_norm2 = x;
    } else if (what == 2) {
      ctrl->est_abs = x;
      ctrl->dots_norm2 = y;
    } else {
      const double s = ctrl->sigma[k];
      double2 h = mk<double2>(x * s, y * s);  // true basis vector k = sigma_k * stored
      if (which == 1) ctrl->h1[k] = h; else ctrl->h2[k] = h;
      ctrl->coef[k] = mk<double2>(h.x * s, h.y * s);
    }
  }
}

static __global__ __launch_bounds__(256) void reduce_partials(const double2 *__restrict__ partial,
                                                        int64_t nblk, Ctrl *__restrict__ ctrl,
                                                        int what, int which) {
  reduce_coef(blockIdx.x, partial, nblk, ctrl, what, which);
}

// Starts a cycle: g = beta e_1, sigma_0.
__device__ inline void cycle_init_dev(Ctrl *ctrl, double beta, double sigma0) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i <= kMaxRestart; i++) ctrl->g[i] = mk<double2>(0, 0);
  ctrl->g[0] = mk<double2>(beta, 0);
  ctrl->sigma[0] = sigma0;
  ctrl->est_abs = beta;
  ctrl->happy = 0;
  ctrl->finite = 1;
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes and the
// final norm, previous rotations applied, new complex Givens rotation
//   rho = sqrt(|a|^2 + |b|^2), c = |a|/rho, s = (a/|a|) conj(b)/rho  (c = 0, s = 1 if a = 0)
// and the rotated right-hand side; |g_{j+1}| is the residual estimate.
__device__ inline void givens_dev(Ctrl *ctrl, int j) {
  if (threadIdx.x != 0) return;
  double2 *col = ctrl->H[j];
  double w0 = 0.0;
  for (int k = 0; k <= j; k++) {
    col[k] = cadd(ctrl->h1[k], ctrl->h2[k]);
    w0 += cabs2(ctrl->h1[k]) + cabs2(ctrl->h2[k]);
  }
  const double hn2 = ctrl->dots_norm2;
  const double hn = sqrt(hn2);
  w0 += hn2;
  col[j + 1] = mk<double2>(hn, 0);
  ctrl->sigma[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
  ctrl->sigma_next = ctrl->sigma[j + 1];
  ctrl->happy = (hn <= 1e-14 * sqrt(w0)) ? 1.0 : 0.0;
  for (int i = 0; i < j; i++) {
    double2 a = col[i], b = col[i + 1], c = ctrl->cs[i], s = ctrl->sn[i];
    col[i] = cadd(cmul(c, a), cmul(s, b));
    col[i + 1] = csub(cmul(c, b), cmul(mk<double2>(s.x, -s.y), a));
  }
  double2 a = col[j], b = col[j + 1];
  const double na = sqrt(cabs2(a));
  const double rho = sqrt(cabs2(a) + cabs2(b));
  double2 c, s;
  if (na == 0.0) {
    c = mk<double2>(0, 0);
    s = mk<double2>(1, 0);
  } else {
    c = mk<double2>(na / rho, 0);
    double2 ph = mk<double2>(a.x / na, a.y / na);
    s = cscale(cmul(ph, mk<double2>(b.x, -b.y)), 1.0 / rho);
  }
  ctrl->cs[j] = c;
  ctrl->sn[j] = s;
  col[j] = cadd(cmul(c, a), cmul(s, b));
  col[j + 1] = mk<double2>(0, 0);
  double2 gj = ctrl->g[j];
  ctrl->g[j] = cmul(c, gj);
  ctrl->g[j + 1] = cmul(mk<double2>(-s.x, s.y), gj);  // -conj(s) g_j
  const double est = sqrt(cabs2(ctrl->g[j + 1]));
  ctrl->est_abs = est;
  ctrl->finite = (isfinite(est) && isfinite(hn)) ? 1.0 : 0.0;
}

// R y = g (k x k upper triangular), then coef_i = sigma_i y_i (flexible:
// coef_i = y_i, the stored preconditioned vectors already carry the scale).
__device__ inline void backsub_dev(Ctrl *ctrl, int k, int flexible) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; i--) {
    double2 s = ctrl->g[i];
    for (int q = i + 1; q < k; q++) s = csub(s, cmul(ctrl->H[q][i], ctrl->y[q]));
    double2 d = ctrl->H[i][i];
    double dd = 1.0 / cabs2(d);
    ctrl->y[i] = cmul(s, mk<double2>(d.x * dd, -d.y * dd));
  }
  for (int i = 0; i < k; i++) ctrl->coef[i] = flexible ? ctrl->y[i] : cscale(ctrl->y[i], ctrl->sigma[i]);
  for (int i = k; i <= kMaxRestart; i++) ctrl->coef[i] = mk<double2>(0, 0);
}

// out[e] (+)= sum_{k < nk} V_k[e] coef[k], accumulated in FP64.
template <typename T, typename TO, bool ACCUM>
__global__ __launch_bounds__(256) void combine(const cx<T> *__restrict__ V, int64_t ldv, int nk,
                                                const double2 *__restrict__ coef,
                                                cx<TO> *__restrict__ out, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double2 acc = ACCUM ? to64(out[e]) : mk<double2>(0, 0);
  for (int k = 0; k < nk; k++) acc = cfma(acc, to64(V[(int64_t)k * ldv + e]), coef[k]);
  out[e] = mk<cx<TO>>((TO)acc.x, (TO)acc.y);
}

// z[e] = s * v[e]
template <typename T>
__global__ __launch_bounds__(256) void scale_copy(const cx<T> *__restrict__ v, double s,
                                                   cx<T> *__restrict__ z, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  z[e] = mk<cx<T>>((T)(v[e].x * s), (T)(v[e].y * s));
}

// x[e] += z[e]
template <typename T>
__global__ __launch_bounds__(256) void add_into64(double2 *__restrict__ x,
                                                   const cx<T> *__restrict__ z, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  x[e] = cadd(x[e], to64(z[e]));
}

// out = (T) (in * s)
template <typename T>
__global__ __launch_bounds__(256) void scale_convert(const double2 *__restrict__ in, double s,
                                                      cx<T> *__restrict__ out, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double2 v = in[e];
  out[e] = mk<cx<T>>((T)(v.x * s), (T)(v.y * s));
}

// z_r = s * Binv_r v_r  (node-block Jacobi)
template <typename T, int NC>
__global__ __launch_bounds__(256) void block_jacobi_apply(const cx<T> *__restrict__ binv,
                                                           const cx<T> *__restrict__ v, T s,
                                                           cx<T> *__restrict__ z, int64_t nrows) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nrows * NC) return;
  const int64_t r = e / NC;
  const int i = (int)(e - r * NC);
  cx<T> acc = mk<cx<T>>(0, 0);
#pragma unroll
  for (int j = 0; j < NC; j++) acc = cfma(acc, binv[(r * NC + i) * NC + j], v[r * NC + j]);
  z[e] = mk<cx<T>>(acc.x * s, acc.y * s);
}

static __global__ void cycle_init(Ctrl *ctrl, double beta, double sigma0) { cycle_init_dev(ctrl, beta, sigma0); }
static __global__ void givens_step(Ctrl *ctrl, int j) { givens_dev(ctrl, j); }
static __global__ void back_substitute(Ctrl *ctrl, int k, int flexible) { backsub_dev(ctrl, k, flexible); }

static __global__ void zero_ctrl(Ctrl *ctrl) {
  double *p = reinterpret_cast<double *>(ctrl);
  const int64_t n = sizeof(Ctrl) / sizeof(double);
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

}  // namespace dst
