// spectral.hpp -- exact inverse of the constant-potential operator on the
// periodic uniform mesh, used as a right preconditioner.
//
// With V replaced by a constant vbar, every spatial 1D factor of the operator
// is circulant, so a discrete Fourier transform over the spatial axes turns
// the system into independent block-tridiagonal systems along time, one per
// spatial mode (block size nc).  For mode theta (per axis th_a = 2 pi k_a / n_a)
// the 1D mass factor has symbol mu_a = h_a (2 + cos th_a)/3 and the 1D
// derivative factor i sin th_a; along time the Galerkin rows are
//   interior  L = -T/2 + h_t S/6,  D = 4 h_t S/6,  U = T/2 + h_t S/6,
//   last      L as above,          D = T/2 + 2 h_t S/6,
// with T = i g0 prod mu_a and
// S = sum_a i g^a (i sin th_a) prod_{b != a} mu_b - (m I + vbar g0) prod mu_a.
// The t = 0 column has been moved to the right-hand side, so the first row
// has no L.  The block systems are solved by block elimination without
// pivoting (pivot inverses precomputed once per solve in FP64).
//
// The discrete transform is computed by direct summation over LDS tiles (any
// axis length).
#pragma once

#include <cmath>

#include "common.hpp"

namespace dst {

struct SpecGeom {
  int d, nc, nt;
  int n[4];          // n[1..d] spatial
  int64_t S;         // modes (= spatial nodes)
  double h[4];       // h[0] = h_t
  double m, vbar;
  double2 g[4][16];  // gamma matrices
  int64_t tw_off[4]; // offsets of per-axis twiddle tables inside the table buffer
};

// Workspace layout of the spectral preconditioner (bytes from its base).
struct SpecLayout {
  size_t piv;    // [nt][S][nc*nc] cx<T> pivot inverses
  size_t tw64;   // double2 twiddles, all axes
  size_t tw32;   // float2 twiddles
  size_t total;
};

inline SpecLayout spec_layout(const dirac_st_problem *p, int prec) {
  SpecLayout L{};
  int64_t S = 1, twn = 0;
  for (int a = 1; a <= p->d; a++) {
    S *= p->n[a];
    twn += p->n[a];
  }
  const size_t cs = prec == 64 ? 16 : 8;
  L.piv = 0;
  L.tw64 = align256(L.piv + (size_t)p->n[0] * S * p->nc * p->nc * cs);
  L.tw32 = align256(L.tw64 + twn * 16);
  L.total = align256(L.tw32 + twn * 8);
  return L;
}

template <int NC, int DS>
__device__ inline void mode_blocks(const SpecGeom &G, int64_t s, const double2 *tw, double2 *L,
                                   double2 *U, double2 *Dint, double2 *Dlast) {
  double mu[DS + 1], sn[DS + 1];
  int64_t t = s;
  double mus = 1.0;
#pragma unroll
  for (int a = 1; a <= DS; a++) {
    const int k = (int)(t % G.n[a]);
    t /= G.n[a];
    const double2 w = tw[G.tw_off[a] + k];  // exp(-i th)
    mu[a] = G.h[a] * (2.0 + w.x) / 3.0;
    sn[a] = -w.y;
    mus *= mu[a];
  }
  const double ht = G.h[0];
#pragma unroll
  for (int q = 0; q < NC * NC; q++) {
    const int i = q / NC, j = q % NC;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int a = 1; a <= DS; a++) {
      double other = 1.0;
#pragma unroll
      for (int b = 1; b <= DS; b++)
        if (b != a) other *= mu[b];
      // i g^a (i sin th_a) other = -g^a sin th_a other
      sr -= G.g[a][q].x * sn[a] * other;
      si -= G.g[a][q].y * sn[a] * other;
    }
    if (i == j) sr -= G.m * mus;
    sr -= G.vbar * G.g[0][q].x * mus;
    si -= G.vbar * G.g[0][q].y * mus;
    // T = i g0 mus
    const double tr = -G.g[0][q].y * mus, ti = G.g[0][q].x * mus;
    L[q] = mk<double2>(-0.5 * tr + ht / 6.0 * sr, -0.5 * ti + ht / 6.0 * si);
    U[q] = mk<double2>(0.5 * tr + ht / 6.0 * sr, 0.5 * ti + ht / 6.0 * si);
    Dint[q] = mk<double2>(4.0 * ht / 6.0 * sr, 4.0 * ht / 6.0 * si);
    Dlast[q] = mk<double2>(0.5 * tr + 2.0 * ht / 6.0 * sr, 0.5 * ti + 2.0 * ht / 6.0 * si);
  }
}

template <int NC>
__device__ inline void matmul_nc(const double2 *a, const double2 *b, double2 *c) {
#pragma unroll
  for (int i = 0; i < NC; i++)
#pragma unroll
    for (int j = 0; j < NC; j++) {
      double2 s = mk<double2>(0, 0);
#pragma unroll
      for (int k = 0; k < NC; k++) s = cfma(s, a[i * NC + k], b[k * NC + j]);
      c[i * NC + j] = s;
    }
}

// Gauss-Jordan inverse with partial pivoting (no conditioning guard); the
// row swap is an unrolled select so the matrix stays in registers.
template <int NC>
__device__ inline void inverse_nc(const double2 *a, double2 *inv) {
  double2 m[NC][2 * NC];
#pragma unroll
  for (int i = 0; i < NC; i++)
#pragma unroll
    for (int j = 0; j < 2 * NC; j++)
      m[i][j] = (j < NC) ? a[i * NC + j] : mk<double2>(j - NC == i ? 1.0 : 0.0, 0.0);
#pragma unroll
  for (int c = 0; c < NC; c++) {
    double best = cabs2(m[c][c]);
    int piv = c;
#pragma unroll
    for (int r = c + 1; r < NC; r++) {
      const double v = cabs2(m[r][c]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
#pragma unroll
    for (int r = c + 1; r < NC; r++) {
      if (r == piv) {
#pragma unroll
        for (int j = 0; j < 2 * NC; j++) {
          double2 t = m[c][j];
          m[c][j] = m[r][j];
          m[r][j] = t;
        }
      }
    }
    double2 d = m[c][c];
    double dd = 1.0 / cabs2(d);
    double2 dinv = mk<double2>(d.x * dd, -d.y * dd);
#pragma unroll
    for (int j = 0; j < 2 * NC; j++) m[c][j] = cmul(m[c][j], dinv);
#pragma unroll
    for (int r = 0; r < NC; r++) {
      if (r == c) continue;
      double2 f = m[r][c];
#pragma unroll
      for (int j = 0; j < 2 * NC; j++) m[r][j] = cfms(m[r][j], f, m[c][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < NC; i++)
#pragma unroll
    for (int j = 0; j < NC; j++) inv[i * NC + j] = m[i][NC + j];
}

// Block elimination along time for every mode, in place on data
// ([nt][S][NC] in the spatial-frequency domain).  One thread per mode; the
// time loop is cut into batches of PF steps whose loads (right-hand side rows
// and pivot inverses) are all issued before the batch's dependent arithmetic,
// so PF memory latencies overlap.
//
// SETUP: the first application after a set-up also computes the pivot
// inverses, P_0 = D, P_tau = D - L P_{tau-1}^{-1} U (the last row with its own
// diagonal block), in FP64 during the forward sweep, stores them rounded to T
// and uses the rounded values exactly as a later application reads them back.
template <typename T, int NC, int DS, bool SETUP>
__global__ __launch_bounds__(64) void spectral_thomas(SpecGeom G, const double2 *__restrict__ tw,
                                                      cx<T> *__restrict__ piv,
                                                      cx<T> *__restrict__ data) {
  using C = cx<T>;
  constexpr int PF = (NC == 2) ? 8 : (sizeof(T) == 4 ? 2 : 1);
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G.S) return;
  double2 L64[NC * NC], U64[NC * NC], Di[NC * NC], Dl[NC * NC];
  mode_blocks<NC, DS>(G, s, tw, L64, U64, Di, Dl);
  C Lm[NC * NC], Um[NC * NC];
#pragma unroll
  for (int q = 0; q < NC * NC; q++) {
    Lm[q] = mk<C>((T)L64[q].x, (T)L64[q].y);
    Um[q] = mk<C>((T)U64[q].x, (T)U64[q].y);
  }
  const int nt = G.nt;
  const int64_t rs = G.S * NC, ps = G.S * NC * NC;
  C *col = data + s * NC;
  C *pcol = piv + s * NC * NC;
  // forward: y_tau = r_tau - L P^{-1}_{tau-1} y_{tau-1}
  C prev[NC];
  if constexpr (SETUP) {
    double2 Pinv[NC * NC];  // P^{-1}_{tau-1} in FP64 (the recurrence)
    C pprev[NC * NC];       // the same rounded to T (what the sweep uses)
    for (int t0 = 0; t0 < nt; t0 += PF) {
      C rb[PF][NC];
#pragma unroll
      for (int u = 0; u < PF; u++) {
        const int tau = t0 + u;
        if (tau < nt) {
#pragma unroll
          for (int i = 0; i < NC; i++) rb[u][i] = col[tau * rs + i];
        }
      }
#pragma unroll
      for (int u = 0; u < PF; u++) {
        const int tau = t0 + u;
        if (tau < nt) {
          const bool last = (tau == nt - 1);
          double2 P[NC * NC], t1[NC * NC], t2[NC * NC], Pn[NC * NC];
          if (tau == 0) {
#pragma unroll
            for (int q = 0; q < NC * NC; q++) P[q] = last ? Dl[q] : Di[q];
          } else {
            matmul_nc<NC>(L64, Pinv, t1);
            matmul_nc<NC>(t1, U64, t2);
#pragma unroll
            for (int q = 0; q < NC * NC; q++) P[q] = csub(last ? Dl[q] : Di[q], t2[q]);
          }
          inverse_nc<NC>(P, Pn);
          if (tau > 0) {
            C z[NC];
#pragma unroll
            for (int i = 0; i < NC; i++) {
              z[i] = mk<C>(0, 0);
#pragma unroll
              for (int j = 0; j < NC; j++) z[i] = cfma(z[i], pprev[i * NC + j], prev[j]);
            }
#pragma unroll
            for (int i = 0; i < NC; i++)
#pragma unroll
              for (int j = 0; j < NC; j++) rb[u][i] = cfms(rb[u][i], Lm[i * NC + j], z[j]);
          }
#pragma unroll
          for (int i = 0; i < NC; i++) {
            col[tau * rs + i] = rb[u][i];
            prev[i] = rb[u][i];
          }
#pragma unroll
          for (int q = 0; q < NC * NC; q++) {
            Pinv[q] = Pn[q];
            pprev[q] = mk<C>((T)Pn[q].x, (T)Pn[q].y);
            pcol[tau * ps + q] = pprev[q];
          }
        }
      }
    }
  } else {
  for (int t0 = 0; t0 < nt; t0 += PF) {
    C rb[PF][NC], pb[PF][NC * NC];
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int tau = t0 + u;
      if (tau < nt) {
#pragma unroll
        for (int i = 0; i < NC; i++) rb[u][i] = col[tau * rs + i];
        if (tau > 0) {
#pragma unroll
          for (int q = 0; q < NC * NC; q++) pb[u][q] = pcol[(tau - 1) * ps + q];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int tau = t0 + u;
      if (tau < nt) {
        if (tau > 0) {
          C z[NC];
#pragma unroll
          for (int i = 0; i < NC; i++) {
            z[i] = mk<C>(0, 0);
#pragma unroll
            for (int j = 0; j < NC; j++) z[i] = cfma(z[i], pb[u][i * NC + j], prev[j]);
          }
#pragma unroll
          for (int i = 0; i < NC; i++)
#pragma unroll
            for (int j = 0; j < NC; j++) rb[u][i] = cfms(rb[u][i], Lm[i * NC + j], z[j]);
        }
#pragma unroll
        for (int i = 0; i < NC; i++) {
          col[tau * rs + i] = rb[u][i];
          prev[i] = rb[u][i];
        }
      }
    }
  }
  }
  // backward: x_tau = P^{-1}_tau (y_tau - U x_{tau+1})
  for (int t0 = nt - 1; t0 >= 0; t0 -= PF) {
    C rb[PF][NC], pb[PF][NC * NC];
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int tau = t0 - u;
      if (tau >= 0) {
#pragma unroll
        for (int i = 0; i < NC; i++) rb[u][i] = col[tau * rs + i];
#pragma unroll
        for (int q = 0; q < NC * NC; q++) pb[u][q] = pcol[tau * ps + q];
      }
    }
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int tau = t0 - u;
      if (tau >= 0) {
        if (tau < nt - 1)
#pragma unroll
          for (int i = 0; i < NC; i++)
#pragma unroll
            for (int j = 0; j < NC; j++) rb[u][i] = cfms(rb[u][i], Um[i * NC + j], prev[j]);
        C x[NC];
#pragma unroll
        for (int i = 0; i < NC; i++) {
          x[i] = mk<C>(0, 0);
#pragma unroll
          for (int j = 0; j < NC; j++) x[i] = cfma(x[i], pb[u][i * NC + j], rb[u][j]);
        }
#pragma unroll
        for (int i = 0; i < NC; i++) {
          col[tau * rs + i] = x[i];
          prev[i] = x[i];
        }
      }
    }
  }
}

// Discrete Fourier transform along one axis by direct summation.
// Element (o, j, q) sits at o * n * stride + j * stride + q, q < stride.
// A workgroup transforms the tile [j = 0..n) x [q = q0, q0 + ti) of one o.
// sign = -1: forward with exp(-2 pi i jk/n); +1: inverse (no 1/n).
// out = scale * transform(in); in and out may be the same buffer.
template <typename T>
__global__ __launch_bounds__(256) void dft_axis(const cx<T> *in, cx<T> *out, int n, int64_t stride,
                                                int ti, int ntile_q, int sign, T scale,
                                                const cx<T> *__restrict__ tw) {
  using C = cx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *tile = reinterpret_cast<C *>(smem_raw);  // [n][ti]
  C *twl = tile + (size_t)n * ti;             // [n]
  const int64_t o = blockIdx.x / ntile_q;
  const int64_t q0 = (int64_t)(blockIdx.x % ntile_q) * ti;
  const int64_t base = o * n * stride + q0;
  for (int t = threadIdx.x; t < n * ti; t += blockDim.x) {
    const int j = t / ti, q = t % ti;
    tile[t] = in[base + (int64_t)j * stride + q];
  }
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    C w = tw[t];
    twl[t] = mk<C>(w.x, sign < 0 ? w.y : -w.y);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n * ti; t += blockDim.x) {
    const int k = t / ti, q = t % ti;
    C acc = mk<C>(0, 0);
    int idx = 0;
    for (int j = 0; j < n; j++) {
      acc = cfma(acc, tile[j * ti + q], twl[idx]);
      idx += k;
      if (idx >= n) idx -= n;
    }
    out[base + (int64_t)k * stride + q] = mk<C>(acc.x * scale, acc.y * scale);
  }
}

// Radix-2 decimation-in-time FFT along one axis of power-of-two length n
// (same element layout and tiling as dft_axis, with a power-of-two tile width
// ti = 2^lti, so every index split is a shift and a mask).  The tile is loaded
// in bit-reversed order into LDS and log2(n) butterfly stages run in place.
template <typename T>
__global__ __launch_bounds__(256) void fft_axis(const cx<T> *in, cx<T> *out, int n, int logn,
                                                int64_t stride, int lti, int ntile_q, int sign,
                                                T scale, const cx<T> *__restrict__ tw) {
  using C = cx<T>;
  extern __shared__ unsigned char smem_raw[];
  const int ti = 1 << lti, qm = ti - 1;
  C *tile = reinterpret_cast<C *>(smem_raw);  // [n][ti]
  C *twl = tile + (size_t)n * ti;             // [n/2]
  const int64_t o = blockIdx.x / ntile_q;
  const int64_t q0 = (int64_t)(blockIdx.x % ntile_q) * ti;
  const int64_t base = o * n * stride + q0;
  for (int t = threadIdx.x; t < n * ti; t += blockDim.x) {
    const int j = t >> lti, q = t & qm;
    const int jr = (int)(__brev((unsigned)j) >> (32 - logn));
    tile[(jr << lti) + q] = in[base + (int64_t)j * stride + q];
  }
  for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
    C w = tw[t];
    twl[t] = mk<C>(w.x, sign < 0 ? w.y : -w.y);
  }
  __syncthreads();
  for (int lh = 0, lstep = n / 2; lh < logn; lh++, lstep >>= 1) {
    // stage with butterfly span half = 2^lh
    const int hm = (1 << lh) - 1;
    for (int t = threadIdx.x; t < (n / 2) * ti; t += blockDim.x) {
      const int q = t & qm, k = t >> lti;
      const int pos = k & hm;
      const int i0 = ((k >> lh) << (lh + 1)) + pos, i1 = i0 + (1 << lh);
      const C w = twl[pos * lstep];
      const C a = tile[(i0 << lti) + q], b = tile[(i1 << lti) + q];
      const C tb = cmul(w, b);
      tile[(i0 << lti) + q] = cadd(a, tb);
      tile[(i1 << lti) + q] = csub(a, tb);
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n * ti; t += blockDim.x) {
    const int k = t >> lti, q = t & qm;
    const C v = tile[(k << lti) + q];
    out[base + (int64_t)k * stride + q] = mk<C>(v.x * scale, v.y * scale);
  }
}

}  // namespace dst
