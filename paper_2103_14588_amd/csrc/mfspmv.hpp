// mfspmv.hpp -- the operator applied without a stored matrix.
//
// The assembled block of row node (tau, i) and column node (tau + o_0, i + o)
// is a sum of products of 1D element integrals (App. A; Sec. 4.3 for the
// potential), so A is a sum of Kronecker products of 1D three-point stencils:
//   A = D_t (x) i g0 M_1..M_d
//     + M_t (x) [ sum_a i g_a M_1..D_a..M_d - m M_1..M_d - g0 P_1 M_2..M_d ]
// with, along a periodic spatial axis of step h (offsets -1, 0, +1),
//   M = (h/6, 2h/3, h/6),  D = (-1/2, 0, 1/2),
// P_1 the potential mass matrix along axis 1 (2-point Gauss per element), and
// along time the same stencils cut at the ends: row tau = 1 has no -1 column
// (the t = 0 node is data), row n_t has only element n_t - 1, so its diagonal
// is M = h/3, D = 1/2.
// One thread computes one row node (all nc components) by applying the 1D
// stencils axis after axis (slowest spatial axis first, then axis 1, then
// time) instead of the 3^(d+1) blocks: about 70 complex-by-real products
// per time offset for 2+1D instead of 4 complex products for each of 27
// stored blocks, and only x is read, once per workgroup tile (LDS), and y
// written: 64 bytes per row in complex128 instead of 1.8 kB.
#pragma once

#include <cmath>

#include "common.hpp"
#include "spmv.hpp"

namespace dst {

struct MfGeom {
  int d, nc, nt;
  int n[4];
  int64_t S;
  double h[4];  // h[0] = h_t
  double m;
  int vkind;
  double v0, x0, lw;
  double2 g[4][16];  // gamma matrices, row-major nc x nc
};

inline MfGeom make_mf_geom(const dirac_st_problem *p) {
  MfGeom G{};
  G.d = p->d;
  G.nc = p->nc;
  G.nt = p->n[0];
  G.S = 1;
  for (int a = 0; a < 4; a++) {
    G.n[a] = a <= p->d ? p->n[a] : 1;
    G.h[a] = a <= p->d ? p->len[a] / p->n[a] : 1.0;
  }
  for (int a = 1; a <= p->d; a++) G.S *= p->n[a];
  G.m = p->m;
  G.vkind = p->vkind;
  G.v0 = p->v0;
  G.x0 = p->x0;
  G.lw = p->lw;
  gamma_set(p->d, G.g);
  return G;
}

__device__ inline double mf_potential(const MfGeom &G, double x) {
  if (G.vkind == DIRAC_ST_V_STEP) return x > G.x0 ? G.v0 : 0.0;
  if (G.vkind == DIRAC_ST_V_SMOOTH) return 0.5 * G.v0 * (1.0 + tanh((x - G.x0) / G.lw));
  return 0.0;
}

// Potential mass row of node i along axis 1: P[i][i-1], P[i][i], P[i][i+1]
// (2-point Gauss-Legendre on the elements i-1 and i, periodic).
__device__ inline void mf_pot_row(const MfGeom &G, int i, double (&pr)[3]) {
  pr[0] = pr[1] = pr[2] = 0.0;
  if (G.vkind == DIRAC_ST_V_NONE) return;
  const int n = G.n[1];
  const double h = G.h[1], r3 = 0.57735026918962576451;
#pragma unroll
  for (int side = 0; side < 2; side++) {
    // side 0: element i-1 (node i is its local 1); side 1: element i (local 0)
    const int e = side ? i : (i == 0 ? n - 1 : i - 1);
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const double xi = 0.5 * (1.0 + (q ? r3 : -r3));
      const double w = 0.5 * h * mf_potential(G, (e + xi) * h);
      const double pi = side ? 1.0 - xi : xi;         // phi of node i
      const double po = side ? xi : 1.0 - xi;         // phi of the other node
      pr[1] += w * pi * pi;
      pr[side ? 2 : 0] += w * pi * po;
    }
  }
}

// Row computation.  X(kt, k1, k2, k3, c) returns component c of the column
// node at time slice kt (0 = first present slice) and sorted spatial offset
// k_a = 0, 1, 2 for -1, 0, +1.
// t0_only: only the coupling of row tau = 1 to the t = 0 slice (the columns
// that were moved to the right-hand side), slice 0 being t = 0.
template <typename T, int NC, int DS, typename Fetch>
__device__ __forceinline__ void mf_row(const MfGeom &G, int tau, int i1, Fetch X, cx<T> (&out)[NC],
                                       bool t0_only = false) {
  using C = cx<T>;
  const int ntime = t0_only ? 1 : (G.nt == 1 ? 1 : ((tau == 1 || tau == G.nt) ? 2 : 3));
  const int o0 = (t0_only || tau >= 2) ? -1 : 0;  // time offset of slice 0
  const bool last = tau == G.nt && !t0_only;
  const T ht = (T)G.h[0];
  T Mx[3], Dd[3] = {(T)-0.5, (T)0, (T)0.5}, My[3], Mz[3], Px[3];
  Mx[0] = Mx[2] = (T)(G.h[1] / 6.0);
  Mx[1] = (T)(2.0 * G.h[1] / 3.0);
  My[0] = My[2] = (T)(G.h[DS >= 2 ? 2 : 1] / 6.0);
  My[1] = (T)(2.0 * G.h[DS >= 2 ? 2 : 1] / 3.0);
  Mz[0] = Mz[2] = (T)(G.h[DS >= 3 ? 3 : 1] / 6.0);
  Mz[1] = (T)(2.0 * G.h[DS >= 3 ? 3 : 1] / 3.0);
  {
    double pr[3];
    mf_pot_row(G, i1, pr);
    Px[0] = (T)pr[0];
    Px[1] = (T)pr[1];
    Px[2] = (T)pr[2];
  }
  // Time-weighted spatial sums of one input component c (the stencils do not
  // mix components): t0 (D_t, mass), tm (M_t, mass), ta[a] (M_t, derivative
  // along axis a + 1), tp (M_t, potential); then the gamma matrices spread
  // them over the output components:
  //   out_i += i g0_ic t0 + sum_a i g(a+1)_ic ta[a] - g0_ic tp - m [i == c] tm
#pragma unroll
  for (int i = 0; i < NC; i++) out[i] = mk<C>(0, 0);
  auto comp = [&](int c) {
      C t0 = mk<C>(0, 0), tm = mk<C>(0, 0), tp = mk<C>(0, 0), ta[DS];
#pragma unroll
      for (int a = 0; a < DS; a++) ta[a] = mk<C>(0, 0);
      for (int kt = 0; kt < ntime; kt++) {
        const int o = o0 + kt;
        const T dt = o == 0 ? (last ? (T)0.5 : (T)0) : (o < 0 ? (T)-0.5 : (T)0.5);
        const T mt = o == 0 ? (last ? ht / (T)3 : (T)2 * ht / (T)3) : ht / (T)6;
        C s0 = mk<C>(0, 0), s1 = mk<C>(0, 0), s2 = mk<C>(0, 0), s3 = mk<C>(0, 0), sp = mk<C>(0, 0);
#pragma unroll
        for (int k1 = 0; k1 < 3; k1++) {
          // U = M_y M_z x, W2 = D_y M_z x, W3 = M_y D_z x at x offset k1
          C U = mk<C>(0, 0), W2 = mk<C>(0, 0), W3 = mk<C>(0, 0);
          if (DS == 1) {
            U = X(kt, k1, 1, 1, c);
          } else {
#pragma unroll
            for (int k2 = 0; k2 < 3; k2++) {
              C a = mk<C>(0, 0), b = mk<C>(0, 0);  // M_z x, D_z x (the node itself for 2+1D)
              if (DS == 2) {
                a = X(kt, k1, k2, 1, c);
              } else {
#pragma unroll
                for (int k3 = 0; k3 < 3; k3++) {
                  const C v = X(kt, k1, k2, k3, c);
                  a.x += Mz[k3] * v.x;
                  a.y += Mz[k3] * v.y;
                  b.x += Dd[k3] * v.x;
                  b.y += Dd[k3] * v.y;
                }
              }
              U.x += My[k2] * a.x;
              U.y += My[k2] * a.y;
              W2.x += Dd[k2] * a.x;
              W2.y += Dd[k2] * a.y;
              if (DS == 3) {
                W3.x += My[k2] * b.x;
                W3.y += My[k2] * b.y;
              }
            }
          }
          // along axis 1
          s0.x += Mx[k1] * U.x;
          s0.y += Mx[k1] * U.y;
          s1.x += Dd[k1] * U.x;
          s1.y += Dd[k1] * U.y;
          sp.x += Px[k1] * U.x;
          sp.y += Px[k1] * U.y;
          if (DS >= 2) {
            s2.x += Mx[k1] * W2.x;
            s2.y += Mx[k1] * W2.y;
          }
          if (DS == 3) {
            s3.x += Mx[k1] * W3.x;
            s3.y += Mx[k1] * W3.y;
          }
        }
        // along time
        t0.x += dt * s0.x;
        t0.y += dt * s0.y;
        tm.x += mt * s0.x;
        tm.y += mt * s0.y;
        tp.x += mt * sp.x;
        tp.y += mt * sp.y;
        ta[0].x += mt * s1.x;
        ta[0].y += mt * s1.y;
        if (DS >= 2) {
          ta[1].x += mt * s2.x;
          ta[1].y += mt * s2.y;
        }
        if (DS == 3) {
          ta[DS - 1].x += mt * s3.x;
          ta[DS - 1].y += mt * s3.y;
        }
      }
      const T m = (T)G.m;
#pragma unroll
      for (int i = 0; i < NC; i++) {
        const double2 g0 = G.g[0][i * NC + c];
        const T gx = (T)g0.x, gy = (T)g0.y;
        T re = -gy * t0.x - gx * t0.y - (gx * tp.x - gy * tp.y);
        T im = -gy * t0.y + gx * t0.x - (gx * tp.y + gy * tp.x);
#pragma unroll
        for (int a = 0; a < DS; a++) {
          const double2 ga = G.g[a + 1][i * NC + c];
          re += -(T)ga.y * ta[a].x - (T)ga.x * ta[a].y;
          im += -(T)ga.y * ta[a].y + (T)ga.x * ta[a].x;
        }
        if (i == c) {
          re -= m * tm.x;
          im -= m * tm.y;
        }
        out[i].x += re;
        out[i].y += im;
      }
  };
  if constexpr (DS == 3) {
    // 4 components x 81 neighbours: one component at a time bounds the registers
#pragma unroll 1
    for (int c = 0; c < NC; c++) comp(c);
  } else {
#pragma unroll
    for (int c = 0; c < NC; c++) comp(c);
  }
}

// 1+1D and 2+1D (nc = 2): a workgroup owns TY x TX row nodes of one time
// node and stages the x values of (present time slices) x (TY + 2) x (TX + 2)
// nodes in LDS, periodic in space.
template <typename T, int DS, bool RESID>
__global__ __launch_bounds__(256) void mf_lds_kernel(MfGeom G, int64_t ntiles, const cx<T> *__restrict__ x,
                                                     const cx<T> *__restrict__ bvec, cx<T> *__restrict__ y,
                                                     T alpha) {
  using C = cx<T>;
  constexpr int NC = 2;
  constexpr int TX = DS == 1 ? 256 : 64, TY = DS == 1 ? 1 : 4;
  constexpr int SX = TX + 2, SY = DS == 1 ? 1 : TY + 2;
  __shared__ C xs[3 * SY * SX * NC];
  const int n1 = G.n[1], n2 = DS == 2 ? G.n[2] : 1;
  const int txt = (n1 + TX - 1) / TX, tyt = (n2 + TY - 1) / TY;
  int64_t t = xcd_tile(blockIdx.x, ntiles);
  const int xb = (int)(t % txt);
  t /= txt;
  const int yb = (int)(t % tyt);
  const int tau = (int)(t / tyt) + 1;
  const int x0 = xb * TX, y0 = yb * TY;
  const int tau0 = tau >= 2 ? tau - 1 : tau;
  const int ntime = G.nt == 1 ? 1 : ((tau == 1 || tau == G.nt) ? 2 : 3);
  for (int e = threadIdx.x; e < ntime * SY * SX * NC; e += 256) {
    const int c = e % NC;
    int node = e / NC;
    const int lx = node % SX;
    node /= SX;
    const int ly = node % SY, kt = node / SY;
    int xg = (x0 - 1 + lx) % n1;  // the tile can be wider than a short axis
    xg += xg < 0 ? n1 : 0;
    int yg = 0;
    if (DS == 2) {
      yg = (y0 - 1 + ly) % n2;
      yg += yg < 0 ? n2 : 0;
    }
    xs[e] = x[((int64_t)(tau0 + kt - 1) * G.S + (int64_t)yg * n1 + xg) * NC + c];
  }
  __syncthreads();
  const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
  const int xg = x0 + lx, yg = y0 + ly;
  if (xg >= n1 || yg >= n2) return;
  auto fetch = [&](int kt, int k1, int k2, int, int c) -> C {
    return xs[((kt * SY + ly + (DS == 2 ? k2 : 0)) * SX + lx + k1) * NC + c];
  };
  C out[NC];
  mf_row<T, NC, DS>(G, tau, xg, fetch, out);
  const int64_t row = (int64_t)(tau - 1) * G.S + (int64_t)yg * n1 + xg;
#pragma unroll
  for (int c = 0; c < NC; c++) {
    const int64_t o = row * NC + c;
    if (RESID) {
      const C bb = bvec[o];
      y[o] = mk<C>(bb.x - out[c].x, bb.y - out[c].y);
    } else {
      y[o] = mk<C>(alpha * out[c].x, alpha * out[c].y);
    }
  }
}

// 3+1D (nc = 4): one thread per row node, neighbours read from global memory
// (L1/L2), 64 consecutive nodes of axis 1 per wavefront.
template <typename T, bool RESID>
__global__ __launch_bounds__(256) void mf_direct_kernel(MfGeom G, int64_t nrows, const cx<T> *__restrict__ x,
                                                        const cx<T> *__restrict__ bvec, cx<T> *__restrict__ y,
                                                        T alpha) {
  using C = cx<T>;
  constexpr int NC = 4;
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= nrows) return;
  const int n1 = G.n[1], n2 = G.n[2], n3 = G.n[3];
  const int tau = (int)(row / G.S) + 1;
  int64_t s = row - (int64_t)(tau - 1) * G.S;
  const int i1 = (int)(s % n1);
  s /= n1;
  const int i2 = (int)(s % n2), i3 = (int)(s / n2);
  const int tau0 = tau >= 2 ? tau - 1 : tau;
  int c1[3], c2[3], c3[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    c1[k] = (i1 + k - 1 + n1) % n1;
    c2[k] = (i2 + k - 1 + n2) % n2;
    c3[k] = (i3 + k - 1 + n3) % n3;
  }
  auto fetch = [&](int kt, int k1, int k2, int k3, int c) -> C {
    const int64_t node = (int64_t)(tau0 + kt - 1) * G.S + ((int64_t)c3[k3] * n2 + c2[k2]) * n1 + c1[k1];
    return x[node * NC + c];
  };
  C out[NC];
  mf_row<T, NC, 3>(G, tau, i1, fetch, out);
#pragma unroll
  for (int c = 0; c < NC; c++) {
    const int64_t o = row * NC + c;
    if (RESID) {
      const C bb = bvec[o];
      y[o] = mk<C>(bb.x - out[c].x, bb.y - out[c].y);
    } else {
      y[o] = mk<C>(alpha * out[c].x, alpha * out[c].y);
    }
  }
}

// b = -D_w21 psi0 (Sec. 2.1): rows of tau = 1 from the t = 0 slice, zero
// elsewhere.  One thread per row, neighbours read from global memory.
template <int NC, int DS>
__global__ __launch_bounds__(256) void mf_rhs_kernel(MfGeom G, int64_t nrows, const double2 *__restrict__ psi0,
                                                     double2 *__restrict__ b) {
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= nrows) return;
  if (row >= G.S) {
#pragma unroll
    for (int c = 0; c < NC; c++) b[row * NC + c] = mk<double2>(0, 0);
    return;
  }
  int ii[3] = {0, 0, 0};
  int64_t s = row;
#pragma unroll
  for (int a = 0; a < DS; a++) {
    ii[a] = (int)(s % G.n[a + 1]);
    s /= G.n[a + 1];
  }
  auto fetch = [&](int, int k1, int k2, int k3, int c) -> double2 {
    const int k[3] = {k1, k2, k3};
    int64_t node = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < DS; a++) {
      const int n = G.n[a + 1];
      node += (int64_t)((ii[a] + k[a] - 1 + n) % n) * stride;
      stride *= n;
    }
    return psi0[node * NC + c];
  };
  double2 out[NC];
  mf_row<double, NC, DS>(G, 1, ii[0], fetch, out, true);
#pragma unroll
  for (int c = 0; c < NC; c++) b[row * NC + c] = mk<double2>(-out[c].x, -out[c].y);
}

inline hipError_t launch_rhs_mf(const dirac_st_problem *p, const void *psi0, void *b, hipStream_t st) {
  const MfGeom G = make_mf_geom(p);
  const int64_t nrows = (int64_t)G.nt * G.S;
  const unsigned g = (unsigned)((nrows + 255) / 256);
  const double2 *in = (const double2 *)psi0;
  double2 *out = (double2 *)b;
  if (G.d == 1) mf_rhs_kernel<2, 1><<<g, 256, 0, st>>>(G, nrows, in, out);
  else if (G.d == 2) mf_rhs_kernel<2, 2><<<g, 256, 0, st>>>(G, nrows, in, out);
  else mf_rhs_kernel<4, 3><<<g, 256, 0, st>>>(G, nrows, in, out);
  return hipGetLastError();
}

// y = alpha A x, or y = b - A x (resid), without a stored matrix.
template <typename T>
inline hipError_t launch_spmv_mf(const dirac_st_problem *p, const void *x, const void *bvec, void *y, T alpha,
                                 bool resid, hipStream_t st) {
  const MfGeom G = make_mf_geom(p);
  const int tk = kt_start(DIRAC_ST_TIMED_SPMV_MF, st);
  if (G.d == 3) {
    const int64_t nrows = (int64_t)G.nt * G.S;
    const unsigned g = (unsigned)((nrows + 255) / 256);
    if (resid)
      mf_direct_kernel<T, true><<<g, 256, 0, st>>>(G, nrows, (const cx<T> *)x, (const cx<T> *)bvec, (cx<T> *)y,
                                                    alpha);
    else
      mf_direct_kernel<T, false><<<g, 256, 0, st>>>(G, nrows, (const cx<T> *)x, (const cx<T> *)bvec, (cx<T> *)y,
                                                     alpha);
  } else {
    const int TX = G.d == 1 ? 256 : 64, TY = G.d == 1 ? 1 : 4;
    const int64_t ntiles = (int64_t)G.nt * ((G.n[1] + TX - 1) / TX) * (G.d == 2 ? (G.n[2] + TY - 1) / TY : 1);
    auto go = [&](auto kern) {
      kern<<<(unsigned)ntiles, 256, 0, st>>>(G, ntiles, (const cx<T> *)x, (const cx<T> *)bvec, (cx<T> *)y, alpha);
    };
    if (G.d == 1) resid ? go(mf_lds_kernel<T, 1, true>) : go(mf_lds_kernel<T, 1, false>);
    else resid ? go(mf_lds_kernel<T, 2, true>) : go(mf_lds_kernel<T, 2, false>);
  }
  kt_stop(tk, st);
  return hipGetLastError();
}

// The solvers' operator: stored blocks (structured or indexed SpMV) or the
// matrix-free stencil of A->prob.
template <typename T>
inline hipError_t apply_op(const dirac_st_bsr *A, bool mf, const void *val, const void *x, const void *bvec,
                           void *y, T alpha, bool resid, hipStream_t st) {
  if (mf) return launch_spmv_mf<T>(&A->prob, x, bvec, y, alpha, resid, st);
  return launch_spmv_st<T>(A, val, x, bvec, y, alpha, resid, st);
}

}  // namespace dst
