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
// Every time slice is reduced once per spatial node to two nc-vectors,
//   S0 = (M_1..M_d) x  and  F = [sum_a i g_a (..D_a..) - m (M..M) - g0 P_1 (M..)] x,
// by applying the 1D stencils axis after axis (about 70 complex-by-real
// products for 2+1D instead of 4 complex products for each of 27 stored
// blocks); row tau then combines the (S0, F) of slices tau - 1, tau, tau + 1
// with the time weights.  A workgroup sweeps a block of consecutive time rows
// so each slice is staged (LDS, for d <= 2) and reduced once; only x is read
// and y written: 64 bytes per row in complex128 instead of 1.8 kB.
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

// Spatial part of one time slice at one node.  X(k1, k2, k3, c) returns
// component c of the slice's node at sorted offsets k_a = 0, 1, 2 (-1, 0, +1)
// along axis a + 1.  Returns
//   S0 = (M_1..M_d) x                                   (feeds D_t (x) i g0)
//   F  = sum_a i g_a (M..D_a..M) x - m S0 - g0 (P_1 M_2..M_d) x   (feeds M_t)
// The stencils act on each input component separately; the gamma matrices
// then spread it over the output components.
template <typename T, int NC, int DS, typename Fetch>
__device__ __forceinline__ void mf_slice(const MfGeom &G, const T (&Mx)[3], const T (&My)[3], const T (&Mz)[3],
                                         const T (&Px)[3], Fetch X, cx<T> (&S0)[NC], cx<T> (&F)[NC]) {
  using C = cx<T>;
  const T Dd[3] = {(T)-0.5, (T)0, (T)0.5};
#pragma unroll
  for (int i = 0; i < NC; i++) S0[i] = F[i] = mk<C>(0, 0);
  auto comp = [&](int c) __attribute__((always_inline)) {
    C s0 = mk<C>(0, 0), s1 = mk<C>(0, 0), s2 = mk<C>(0, 0), s3 = mk<C>(0, 0), sp = mk<C>(0, 0);
#pragma unroll
    for (int k1 = 0; k1 < 3; k1++) {
      // U = M_y M_z x, W2 = D_y M_z x, W3 = M_y D_z x at axis-1 offset k1
      C U = mk<C>(0, 0), W2 = mk<C>(0, 0), W3 = mk<C>(0, 0);
      if (DS == 1) {
        U = X(k1, 1, 1, c);
      } else {
#pragma unroll
        for (int k2 = 0; k2 < 3; k2++) {
          C a = mk<C>(0, 0), b = mk<C>(0, 0);  // M_z x, D_z x (the node itself for 2+1D)
          if (DS == 2) {
            a = X(k1, k2, 1, c);
          } else {
#pragma unroll
            for (int k3 = 0; k3 < 3; k3++) {
              const C v = X(k1, k2, k3, c);
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
    const C sa[3] = {s1, s2, s3};
    const T m = (T)G.m;
#pragma unroll
    for (int i = 0; i < NC; i++) {
      const double2 g0 = G.g[0][i * NC + c];
      // - g0 sp
      T re = -((T)g0.x * sp.x - (T)g0.y * sp.y), im = -((T)g0.x * sp.y + (T)g0.y * sp.x);
#pragma unroll
      for (int a = 0; a < DS; a++) {
        const double2 ga = G.g[a + 1][i * NC + c];
        // i g_a sa = (-gy + i gx) sa
        re += -(T)ga.y * sa[a].x - (T)ga.x * sa[a].y;
        im += -(T)ga.y * sa[a].y + (T)ga.x * sa[a].x;
      }
      if (i == c) {
        re -= m * s0.x;
        im -= m * s0.y;
        S0[i] = s0;
      }
      F[i].x += re;
      F[i].y += im;
    }
  };
  if constexpr (DS == 3) {
    // 4 components x 27 neighbours: one component at a time bounds the registers
#pragma unroll 1
    for (int c = 0; c < NC; c++) comp(c);
  } else {
#pragma unroll
    for (int c = 0; c < NC; c++) comp(c);
  }
}

// Spatial stencil coefficients of the thread's node (axis-1 index i1).
template <typename T, int DS>
__device__ __forceinline__ void mf_coeffs(const MfGeom &G, int i1, T (&Mx)[3], T (&My)[3], T (&Mz)[3],
                                          T (&Px)[3]) {
  const double hs[3] = {G.h[1], G.h[DS >= 2 ? 2 : 1], G.h[DS >= 3 ? 3 : 1]};
  Mx[0] = Mx[2] = (T)(hs[0] / 6.0);
  Mx[1] = (T)(2.0 * hs[0] / 3.0);
  My[0] = My[2] = (T)(hs[1] / 6.0);
  My[1] = (T)(2.0 * hs[1] / 3.0);
  Mz[0] = Mz[2] = (T)(hs[2] / 6.0);
  Mz[1] = (T)(2.0 * hs[2] / 3.0);
  double pr[3];
  mf_pot_row(G, i1, pr);
#pragma unroll
  for (int k = 0; k < 3; k++) Px[k] = (T)pr[k];
}

// Row tau from the slices tau - 1 (a2, absent for tau = 1), tau (a1) and
// tau + 1 (a0, absent for tau = n_t):
//   out = sum_o D_t(tau, o) i g0 S0(tau + o) + M_t(tau, o) F(tau + o).
template <typename T, int NC>
__device__ __forceinline__ void mf_time(const MfGeom &G, int tau, const cx<T> (&S2)[NC], const cx<T> (&F2)[NC],
                                        const cx<T> (&S1)[NC], const cx<T> (&F1)[NC], const cx<T> (&S0)[NC],
                                        const cx<T> (&F0)[NC], cx<T> (&out)[NC]) {
  using C = cx<T>;
  const T h = (T)G.h[0];
  const bool first = tau == 1, last = tau == G.nt;
  // time weights of the offsets -1, 0, +1
  const T dm = first ? (T)0 : (T)-0.5, mm = first ? (T)0 : h / (T)6;
  const T dz = last ? (T)0.5 : (T)0, mz = last ? h / (T)3 : (T)2 * h / (T)3;
  const T dp = last ? (T)0 : (T)0.5, mp = last ? (T)0 : h / (T)6;
  C sd[NC];
#pragma unroll
  for (int j = 0; j < NC; j++) {
    sd[j].x = dz * S1[j].x;
    sd[j].y = dz * S1[j].y;
    out[j].x = mz * F1[j].x;
    out[j].y = mz * F1[j].y;
    if (!first) {
      sd[j].x += dm * S2[j].x;
      sd[j].y += dm * S2[j].y;
      out[j].x += mm * F2[j].x;
      out[j].y += mm * F2[j].y;
    }
    if (!last) {
      sd[j].x += dp * S0[j].x;
      sd[j].y += dp * S0[j].y;
      out[j].x += mp * F0[j].x;
      out[j].y += mp * F0[j].y;
    }
  }
#pragma unroll
  for (int i = 0; i < NC; i++)
#pragma unroll
    for (int j = 0; j < NC; j++) {
      const double2 g0 = G.g[0][i * NC + j];
      if (g0.x == 0.0 && g0.y == 0.0) continue;
      // i g0 sd = (-gy + i gx) sd
      out[i].x += -(T)g0.y * sd[j].x - (T)g0.x * sd[j].y;
      out[i].y += -(T)g0.y * sd[j].y + (T)g0.x * sd[j].x;
    }
}

template <typename T, int NC, bool RESID>
__device__ __forceinline__ void mf_store(int64_t row, const cx<T> (&out)[NC], const cx<T> *__restrict__ bvec,
                                         cx<T> *__restrict__ y, T alpha) {
#pragma unroll
  for (int c = 0; c < NC; c++) {
    const int64_t o = row * NC + c;
    if (RESID) {
      const cx<T> bb = bvec[o];
      y[o] = mk<cx<T>>(bb.x - out[c].x, bb.y - out[c].y);
    } else {
      y[o] = mk<cx<T>>(alpha * out[c].x, alpha * out[c].y);
    }
  }
}

// Time-blocked sweep (the 3+1D kernel; the LDS kernel spells the same loop
// out around its staging): the slices tau_a - 1 .. tau_b + 1
// (those that exist) in order, each reduced once to (S0, F) at the node, kept
// in a three-slice window; row tau is written as soon as slice tau + 1 (or,
// for the last row, slice n_t) is done.  Every slice is read and reduced once
// instead of three times.  SLICE(sigma, S0, F) computes slice sigma;
// NEXT(sigma) is called before it with the slice that follows (staging).
template <typename T, int NC, bool RESID, typename Slice, typename Next>
__device__ __forceinline__ void mf_sweep(const MfGeom &G, int tau_a, int tau_b, bool own, int64_t node,
                                         Slice slice, Next next, const cx<T> *__restrict__ bvec,
                                         cx<T> *__restrict__ y, T alpha) {
  using C = cx<T>;
  const int s0 = tau_a >= 2 ? tau_a - 1 : 1, s1 = tau_b < G.nt ? tau_b + 1 : G.nt;
  C A0[NC], B0[NC], A1[NC], B1[NC], A2[NC], B2[NC];  // (S0, F) of slices sigma, sigma-1, sigma-2
#pragma unroll
  for (int c = 0; c < NC; c++) A0[c] = B0[c] = A1[c] = B1[c] = mk<C>(0, 0);
  for (int sg = s0; sg <= s1; sg++) {
    next(sg);
#pragma unroll
    for (int c = 0; c < NC; c++) {
      A2[c] = A1[c];
      B2[c] = B1[c];
      A1[c] = A0[c];
      B1[c] = B0[c];
    }
    slice(sg, A0, B0);
    const int tau = sg - 1;  // complete once slice tau + 1 is in
    if (own && tau >= tau_a && tau <= tau_b) {
      C out[NC];
      mf_time<T, NC>(G, tau, A2, B2, A1, B1, A0, B0, out);
      mf_store<T, NC, RESID>((int64_t)(tau - 1) * G.S + node, out, bvec, y, alpha);
    }
  }
  if (own && tau_b == G.nt) {  // the last row has no slice after it
    C out[NC];
    mf_time<T, NC>(G, G.nt, A1, B1, A0, B0, A0, B0, out);
    mf_store<T, NC, RESID>((int64_t)(G.nt - 1) * G.S + node, out, bvec, y, alpha);
  }
}

// 1+1D and 2+1D (nc = 2): a workgroup owns TY x TX nodes of axes 2 x 1 and
// TT consecutive time rows; each slice of (TY + 2) x (TX + 2) nodes (periodic
// halo) is staged in LDS, double buffered: the next slice's global loads are
// in flight while the current one is reduced.
template <typename T, int DS, bool RESID>
__global__ __launch_bounds__(256) void mf_tb_kernel(MfGeom G, int TT, int64_t ntiles, const cx<T> *__restrict__ x,
                                                    const cx<T> *__restrict__ bvec, cx<T> *__restrict__ y,
                                                    T alpha) {
  using C = cx<T>;
  constexpr int NC = 2;
  constexpr int TX = DS == 1 ? 256 : 64, TY = DS == 1 ? 1 : 4;
  constexpr int SX = TX + 2, SY = DS == 1 ? 1 : TY + 2;
  constexpr int SL = SY * SX * NC, PER = (SL + 255) / 256;
  __shared__ C xs[2][SL];
  const int n1 = G.n[1], n2 = DS == 2 ? G.n[2] : 1;
  const int txt = (n1 + TX - 1) / TX, tyt = (n2 + TY - 1) / TY;
  int64_t t = xcd_tile(blockIdx.x, ntiles);
  const int xb = (int)(t % txt);
  t /= txt;
  const int yb = (int)(t % tyt);
  const int tb = (int)(t / tyt);
  const int x0 = xb * TX, y0 = yb * TY;
  const int tau_a = tb * TT + 1, tau_b = min(tau_a + TT - 1, G.nt);
  // staged element e of a slice -> its offset inside the slice
  int64_t goff[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int e = threadIdx.x + 256 * q;
    goff[q] = -1;
    if (e < SL) {
      const int c = e % NC, nd = e / NC, lx = nd % SX, ly = nd / SX;
      int xg = (x0 - 1 + lx) % n1;  // the tile can be wider than a short axis
      xg += xg < 0 ? n1 : 0;
      int yg = 0;
      if (DS == 2) {
        yg = (y0 - 1 + ly) % n2;
        yg += yg < 0 ? n2 : 0;
      }
      goff[q] = ((int64_t)yg * n1 + xg) * NC + c;
    }
  }
  const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
  const int xg = x0 + lx, yg = y0 + ly;
  const bool own = xg < n1 && yg < n2;
  T Mx[3], My[3], Mz[3], Px[3];
  mf_coeffs<T, DS>(G, own ? xg : 0, Mx, My, Mz, Px);
  const int s0 = tau_a >= 2 ? tau_a - 1 : 1, s1 = tau_b < G.nt ? tau_b + 1 : G.nt;
  const int64_t node = (int64_t)yg * n1 + xg;
  C reg[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    reg[q] = mk<C>(0, 0);
    if (goff[q] >= 0) reg[q] = x[(int64_t)(s0 - 1) * G.S * NC + goff[q]];
  }
#pragma unroll
  for (int q = 0; q < PER; q++)
    if (goff[q] >= 0) xs[0][threadIdx.x + 256 * q] = reg[q];
  __syncthreads();
  C A0[NC], B0[NC], A1[NC], B1[NC], A2[NC], B2[NC];  // (S0, F) of slices sg, sg-1, sg-2
#pragma unroll
  for (int c = 0; c < NC; c++) A0[c] = B0[c] = A1[c] = B1[c] = mk<C>(0, 0);
  int buf = 0;
  for (int sg = s0; sg <= s1; sg++) {
    // the next slice's loads are in flight while this one is reduced
    if (sg < s1) {
      const C *xsl = x + (int64_t)sg * G.S * NC;
#pragma unroll
      for (int q = 0; q < PER; q++)
        if (goff[q] >= 0) reg[q] = xsl[goff[q]];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) {
      A2[c] = A1[c];
      B2[c] = B1[c];
      A1[c] = A0[c];
      B1[c] = B0[c];
    }
    if (own) {
      const C *b = xs[buf];
      auto fetch = [&](int k1, int k2, int, int c) __attribute__((always_inline)) -> C {
        return b[((ly + (DS == 2 ? k2 : 0)) * SX + lx + k1) * NC + c];
      };
      mf_slice<T, NC, DS>(G, Mx, My, Mz, Px, fetch, A0, B0);
      const int tau = sg - 1;  // complete once slice tau + 1 is in
      if (tau >= tau_a && tau <= tau_b) {
        C out[NC];
        mf_time<T, NC>(G, tau, A2, B2, A1, B1, A0, B0, out);
        mf_store<T, NC, RESID>((int64_t)(tau - 1) * G.S + node, out, bvec, y, alpha);
      }
    }
    if (sg < s1) {
#pragma unroll
      for (int q = 0; q < PER; q++)
        if (goff[q] >= 0) xs[buf ^ 1][threadIdx.x + 256 * q] = reg[q];
      __syncthreads();
      buf ^= 1;
    }
  }
  if (own && tau_b == G.nt) {  // the last row has no slice after it
    C out[NC];
    mf_time<T, NC>(G, G.nt, A1, B1, A0, B0, A0, B0, out);
    mf_store<T, NC, RESID>((int64_t)(G.nt - 1) * G.S + node, out, bvec, y, alpha);
  }
}

// 3+1D (nc = 4): one thread per spatial node and TT consecutive time rows;
// neighbours read from global memory (L1/L2), 64 consecutive nodes of axis
// 1 per wavefront.
template <typename T, bool RESID>
__global__ __launch_bounds__(256) void mf_tb3_kernel(MfGeom G, int TT, int64_t nthreads,
                                                     const cx<T> *__restrict__ x, const cx<T> *__restrict__ bvec,
                                                     cx<T> *__restrict__ y, T alpha) {
  using C = cx<T>;
  constexpr int NC = 4;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= nthreads) return;
  const int tb = (int)(gid / G.S);
  const int64_t node = gid - (int64_t)tb * G.S;
  const int n1 = G.n[1], n2 = G.n[2], n3 = G.n[3];
  int64_t s = node;
  const int i1 = (int)(s % n1);
  s /= n1;
  const int i2 = (int)(s % n2), i3 = (int)(s / n2);
  int64_t c1[3], c23[3][3];
#pragma unroll
  for (int k = 0; k < 3; k++) c1[k] = (i1 + k - 1 + n1) % n1;
#pragma unroll
  for (int k2 = 0; k2 < 3; k2++)
#pragma unroll
    for (int k3 = 0; k3 < 3; k3++)
      c23[k2][k3] = ((int64_t)((i3 + k3 - 1 + n3) % n3) * n2 + (i2 + k2 - 1 + n2) % n2) * n1;
  T Mx[3], My[3], Mz[3], Px[3];
  mf_coeffs<T, 3>(G, i1, Mx, My, Mz, Px);
  const int tau_a = tb * TT + 1, tau_b = min(tau_a + TT - 1, G.nt);
  auto next = [&](int) {};
  auto slice = [&](int sg, C (&S0)[NC], C (&F)[NC]) __attribute__((always_inline)) {
    const C *xsl = x + (int64_t)(sg - 1) * G.S * NC;
    auto fetch = [&](int k1, int k2, int k3, int c) -> C { return xsl[(c23[k2][k3] + c1[k1]) * NC + c]; };
    mf_slice<T, NC, 3>(G, Mx, My, Mz, Px, fetch, S0, F);
  };
  mf_sweep<T, NC, RESID>(G, tau_a, tau_b, true, node, slice, next, bvec, y, alpha);
}

// b = -D_w21 psi0 (Sec. 2.1): rows of tau = 1 from the t = 0 slice (time
// weights of offset -1: D_t = -1/2, M_t = h_t/6), zero elsewhere.  One
// thread per row, neighbours read from global memory.
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
  auto fetch = [&](int k1, int k2, int k3, int c) -> double2 {
    const int k[3] = {k1, k2, k3};
    int64_t nd = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < DS; a++) {
      const int n = G.n[a + 1];
      nd += (int64_t)((ii[a] + k[a] - 1 + n) % n) * stride;
      stride *= n;
    }
    return psi0[nd * NC + c];
  };
  double Mx[3], My[3], Mz[3], Px[3];
  mf_coeffs<double, DS>(G, ii[0], Mx, My, Mz, Px);
  double2 S0[NC], F[NC];
  mf_slice<double, NC, DS>(G, Mx, My, Mz, Px, fetch, S0, F);
  const double h = G.h[0];
#pragma unroll
  for (int i = 0; i < NC; i++) {
    double re = h / 6.0 * F[i].x, im = h / 6.0 * F[i].y;
#pragma unroll
    for (int j = 0; j < NC; j++) {
      const double2 g0 = G.g[0][i * NC + j];
      // -1/2 i g0 S0
      re += 0.5 * (g0.y * S0[j].x + g0.x * S0[j].y);
      im += 0.5 * (g0.y * S0[j].y - g0.x * S0[j].x);
    }
    b[row * NC + i] = mk<double2>(-re, -im);
  }
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

// time rows per workgroup (per thread for 3+1D): enough workgroups to fill
// the chip, each slice re-read at most (TT + 2) / TT times
inline int mf_time_block(const MfGeom &G) { return G.d == 3 ? 4 : 8; }

// y = alpha A x, or y = b - A x (resid), without a stored matrix.
template <typename T>
inline hipError_t launch_spmv_mf(const dirac_st_problem *p, const void *x, const void *bvec, void *y, T alpha,
                                 bool resid, hipStream_t st) {
  const MfGeom G = make_mf_geom(p);
  const int TT = mf_time_block(G);
  const int64_t tblocks = (G.nt + TT - 1) / TT;
  const int tk = kt_start(DIRAC_ST_TIMED_SPMV_MF, st);
  const cx<T> *xx = (const cx<T> *)x, *bb = (const cx<T> *)bvec;
  cx<T> *yy = (cx<T> *)y;
  if (G.d == 3) {
    const int64_t nth = tblocks * G.S;
    const unsigned g = (unsigned)((nth + 255) / 256);
    if (resid) mf_tb3_kernel<T, true><<<g, 256, 0, st>>>(G, TT, nth, xx, bb, yy, alpha);
    else mf_tb3_kernel<T, false><<<g, 256, 0, st>>>(G, TT, nth, xx, bb, yy, alpha);
  } else {
    const int TX = G.d == 1 ? 256 : 64, TY = G.d == 1 ? 1 : 4;
    const int64_t ntiles = tblocks * ((G.n[1] + TX - 1) / TX) * (G.d == 2 ? (G.n[2] + TY - 1) / TY : 1);
    auto go = [&](auto kern) { kern<<<(unsigned)ntiles, 256, 0, st>>>(G, TT, ntiles, xx, bb, yy, alpha); };
    if (G.d == 1) resid ? go(mf_tb_kernel<T, 1, true>) : go(mf_tb_kernel<T, 1, false>);
    else resid ? go(mf_tb_kernel<T, 2, true>) : go(mf_tb_kernel<T, 2, false>);
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
