// precond.hpp -- the base preconditioners M of right-preconditioned GMRES
// (Sec. 2.2): node-block Jacobi (inverses of the diagonal nc x nc blocks) and
// the spatial-Fourier preconditioner (the operator with the potential replaced
// by a constant, inverted exactly: DFT over every periodic spatial axis, one
// block-tridiagonal solve in time per Fourier mode, inverse DFT).
#pragma once

#include <cmath>

#include "common.hpp"
#include "krylov.hpp"
#include "spectral.hpp"

namespace dst {

static inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// ------------------------------------------------------------ preconditioner
struct Precond {
  int kind = DIRAC_ST_PC_NONE;
  int prec = 64;
  const dirac_st_bsr *A = nullptr;
  // spectral
  SpecGeom G{};
  unsigned char *spec = nullptr;
  SpecLayout SL{};
  // learned correction z += s N(v / s) (flexible GMRES only)
  const dirac_st_nn *nn = nullptr;
  bool nn_on = false;
  unsigned char *nnwork = nullptr;
};

static void spec_geom(const dirac_st_problem *p, double vbar, SpecGeom &G) {
  G = SpecGeom{};
  G.d = p->d;
  G.nc = p->nc;
  G.nt = p->n[0];
  G.S = 1;
  int64_t off = 0;
  for (int a = 0; a < 4; a++) {
    G.n[a] = (a <= p->d) ? p->n[a] : 1;
    G.h[a] = (a <= p->d) ? p->len[a] / p->n[a] : 1.0;
    G.tw_off[a] = 0;
  }
  for (int a = 1; a <= p->d; a++) {
    G.S *= p->n[a];
    G.tw_off[a] = off;
    off += p->n[a];
  }
  G.m = p->m;
  G.vbar = vbar;
  for (int mu = 0; mu < 4; mu++)
    for (int q = 0; q < 16; q++) G.g[mu][q] = mk<double2>(0, 0);
  if (p->d <= 2) {
    G.g[0][0] = mk<double2>(1, 0);
    G.g[0][3] = mk<double2>(-1, 0);
    G.g[1][1] = mk<double2>(1, 0);
    G.g[1][2] = mk<double2>(-1, 0);
    G.g[2][1] = mk<double2>(0, -1);
    G.g[2][2] = mk<double2>(0, -1);
  } else {
    for (int q = 0; q < 4; q++) G.g[0][q * 5] = mk<double2>(q < 2 ? 1 : -1, 0);
    const double2 P[3][4] = {
        {mk<double2>(0, 0), mk<double2>(1, 0), mk<double2>(1, 0), mk<double2>(0, 0)},
        {mk<double2>(0, 0), mk<double2>(0, -1), mk<double2>(0, 1), mk<double2>(0, 0)},
        {mk<double2>(1, 0), mk<double2>(0, 0), mk<double2>(0, 0), mk<double2>(-1, 0)}};
    for (int k = 1; k <= 3; k++)
      for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
          double2 s = P[k - 1][a * 2 + b];
          G.g[k][a * 4 + b + 2] = s;
          G.g[k][(a + 2) * 4 + b] = mk<double2>(-s.x, -s.y);
        }
  }
}

// Twiddles exp(-2 pi i q / n_a) of every spatial axis, FP64 and FP32 copies.
static int spec_twiddles(const SpecGeom &G, unsigned char *base, const SpecLayout &L, hipStream_t s) {
  int64_t tot = 0;
  for (int a = 1; a <= G.d; a++) tot += G.n[a];
  double2 h64[3 * 4096];
  float2 h32[3 * 4096];
  DST_CHECK(tot <= 3 * 4096, "axis too long for the spectral preconditioner");
  for (int a = 1; a <= G.d; a++)
    for (int q = 0; q < G.n[a]; q++) {
      const double th = 2.0 * M_PI * (double)q / (double)G.n[a];
      h64[G.tw_off[a] + q] = mk<double2>(cos(th), -sin(th));
      h32[G.tw_off[a] + q] = mk<float2>((float)cos(th), (float)-sin(th));
    }
  DST_HIP(hipMemcpyAsync(base + L.tw64, h64, tot * sizeof(double2), hipMemcpyHostToDevice, s));
  DST_HIP(hipMemcpyAsync(base + L.tw32, h32, tot * sizeof(float2), hipMemcpyHostToDevice, s));
  // the host arrays live on this stack frame: wait for the copies
  DST_HIP(hipStreamSynchronize(s));
  return 0;
}

template <typename T>
static int pc_setup(Precond &P, const dirac_st_bsr *A, int kind, double vbar, unsigned char *spec,
                    hipStream_t s) {
  P.kind = kind;
  P.prec = sizeof(T) == 8 ? 64 : 32;
  P.A = A;
  if (kind == DIRAC_ST_PC_BLOCK_JACOBI) {
    DST_CHECK((sizeof(T) == 8 ? A->bjinv64 : A->bjinv32) != nullptr,
              "block-Jacobi preconditioner needs bjinv%d", P.prec);
  }
  if (kind != DIRAC_ST_PC_SPECTRAL) return 0;
  P.spec = spec;
  P.SL = spec_layout(&A->prob, P.prec);
  spec_geom(&A->prob, vbar, P.G);
  if (int rc = spec_twiddles(P.G, spec, P.SL, s)) return rc;
  const unsigned g = (unsigned)((P.G.S + 63) / 64);
  const double2 *tw64 = (const double2 *)(spec + P.SL.tw64);
  cx<T> *piv = (cx<T> *)(spec + P.SL.piv);
  if (A->prob.d == 1)
    spectral_setup<T, 2, 1><<<g, 64, 0, s>>>(P.G, tw64, piv);
  else if (A->prob.d == 2)
    spectral_setup<T, 2, 2><<<g, 64, 0, s>>>(P.G, tw64, piv);
  else
    spectral_setup<T, 4, 3><<<g, 64, 0, s>>>(P.G, tw64, piv);
  DST_LAUNCHED();
  return 0;
}

// z = scale * M^{-1} v with the base preconditioner (v, z must differ)
template <typename T>
static int pc_apply_base(const Precond &P, const cx<T> *v, cx<T> *z, double scale, int64_t N,
                         hipStream_t s) {
  const dirac_st_bsr *A = P.A;
  if (P.kind == DIRAC_ST_PC_BLOCK_JACOBI) {
    const cx<T> *binv = (const cx<T> *)(sizeof(T) == 8 ? A->bjinv64 : A->bjinv32);
    if (A->nc == 2)
      block_jacobi_apply<T, 2><<<nblocks(N), 256, 0, s>>>(binv, v, (T)scale, z, A->nrows);
    else
      block_jacobi_apply<T, 4><<<nblocks(N), 256, 0, s>>>(binv, v, (T)scale, z, A->nrows);
    DST_LAUNCHED();
    return 0;
  }
  if (P.kind == DIRAC_ST_PC_SPECTRAL) {
    const SpecGeom &G = P.G;
    const cx<T> *tw = (const cx<T> *)(P.spec + (sizeof(T) == 8 ? P.SL.tw64 : P.SL.tw32));
    const int nc = G.nc;
    int64_t stride = nc;
    const int64_t total = G.S * G.nt * nc;
    // forward transforms, axis 1 first (v -> z), then in place
    for (int pass = 0; pass < 2; pass++) {
      stride = nc;
      for (int a = 1; a <= G.d; a++) {
        const int n = G.n[a];
        const int64_t outer = total / ((int64_t)n * stride);
        int ti = (int)(stride < 2048 / n ? stride : 2048 / n);
        if (ti < 1) ti = 1;
        while (stride % ti) ti--;
        const int ntq = (int)(stride / ti);
        const size_t sh = ((size_t)n * ti + n) * sizeof(cx<T>);
        const bool first = (pass == 0 && a == 1);
        const bool last = (pass == 1 && a == G.d);
        const T sc = last ? (T)(scale / (double)G.S) : (T)1;
        if ((n & (n - 1)) == 0) {
          int logn = 0;
          while ((1 << logn) < n) logn++;
          fft_axis<T><<<(unsigned)(outer * ntq), 256, sh, s>>>(first ? v : z, z, n, logn, stride, ti,
                                                              ntq, pass == 0 ? -1 : 1, sc,
                                                              tw + G.tw_off[a]);
        } else {
          dft_axis<T><<<(unsigned)(outer * ntq), 256, sh, s>>>(first ? v : z, z, n, stride, ti, ntq,
                                                              pass == 0 ? -1 : 1, sc,
                                                              tw + G.tw_off[a]);
        }
        DST_LAUNCHED();
        stride *= n;
      }
      if (pass == 0) {
        const unsigned g = (unsigned)((G.S + 63) / 64);
        const double2 *tw64 = (const double2 *)(P.spec + P.SL.tw64);
        const cx<T> *piv = (const cx<T> *)(P.spec + P.SL.piv);
        if (G.d == 1)
          spectral_thomas<T, 2, 1><<<g, 64, 0, s>>>(G, tw64, piv, z);
        else if (G.d == 2)
          spectral_thomas<T, 2, 2><<<g, 64, 0, s>>>(G, tw64, piv, z);
        else
          spectral_thomas<T, 4, 3><<<g, 64, 0, s>>>(G, tw64, piv, z);
        DST_LAUNCHED();
      }
    }
    return 0;
  }
  set_error("no preconditioner to apply");
  return DIRAC_ST_EINVAL;
}

}  // namespace dst
