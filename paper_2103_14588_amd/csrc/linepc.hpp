// linepc.hpp -- exact inverse of the operator for potentials that depend on
// the first spatial coordinate only, used as a right preconditioner.
//
// Every potential of the method (none, the step of Sec. 4.3, its smooth
// version) depends on x = x_1 only, so the operator is a sum of Kronecker
// products of 1D factors:
//   A = D_t (x) X0 + M_t (x) X1,
//   X0 = i g0 M_x M_y M_z,
//   X1 = i g1 D_x M_y M_z + i g2 M_x D_y M_z + i g3 M_x M_y D_z
//        - m M_x M_y M_z - g0 P_x M_y M_z,
// with P_x the 1D potential mass matrix (2-point Gauss per element, as in the
// assembly).  Three exact reductions:
//   time    D_t = M_t W diag(lambda) W^{-1}: apply Q = W^{-1} M_t^{-1} along
//           t, solve one spatial problem per eigenvalue, apply W along t;
//   y, z    periodic circulant factors: a DFT turns M_a into
//           mu_a = h_a (2 + cos th_a) / 3 and D_a into i sin th_a;
//   x       what is left per (lambda, k_y, k_z) is a periodic block
//           tridiagonal system along x with nc x nc blocks
//             L_i = (h/6) C_M - C_D/2 - P[i][i-1] C_P,
//             D_i = (2h/3) C_M       - P[i][i]   C_P,
//             U_i = (h/6) C_M + C_D/2 - P[i][i+1] C_P,
//           C_M = i lambda mu g0 - m mu + sum_a i g_a (i sin th_a) prod_{b != a} mu_b,
//           C_D = i mu g1, C_P = mu g0, mu = prod over the transverse axes,
//           solved by block elimination with a border for the periodic
//           coupling (factors precomputed once per operator, in FP64).
// Apply: tgemm(Q) -> DFT(y, z) -> line_solve -> inverse DFT -> tgemm(W).
#pragma once

#include <cmath>

#include "common.hpp"
#include "spectral.hpp"

namespace dst {

// Workspace layout of the line preconditioner (bytes from its base).
struct LineLayout {
  size_t tw64, tw32, lam, q64, w64, q32, w32, pot, fac, lined, flag, buf, buf2, total;
  // DFT matrices of the transverse axes a = 2, 3 (forward F, inverse F^{-1}),
  // padded to dpm[a] x dpk[a]
  size_t f64[4], fi64[4], f32[4], fi32[4];
  int dpm[4], dpk[4];
  int pm, pk;      // Q and W padded to pm x pk (multiples of 64 and 16), zero filled
  int64_t lines;   // n_t * (spatial nodes / n_1)
  int slabs, tl;   // time slabs and rows per slab (tl x tl time factors)
};

// slabs = 1: the whole time interval; slabs > 1: the time-slab decomposition,
// every slab the same tl = n_t / slabs rows (the caller checks divisibility)
inline LineLayout line_layout(const dirac_st_problem *p, int prec, int slabs = 1) {
  LineLayout L{};
  const int nt = p->n[0], nc = p->nc;
  L.slabs = slabs;
  L.tl = nt / slabs;
  int64_t S = 1, twn = 0;
  for (int a = 1; a <= p->d; a++) {
    S *= p->n[a];
    twn += p->n[a];
  }
  L.lines = (int64_t)nt * (S / p->n[1]);
  L.pm = (L.tl + 63) / 64 * 64;
  L.pk = (L.tl + 15) / 16 * 16;
  const size_t cs = prec == 64 ? 16 : 8;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t r = off;
    off += align256(b);
    return r;
  };
  L.tw64 = take(twn * 16);
  L.tw32 = take(twn * 8);
  L.lam = take((size_t)nt * 16);
  L.q64 = take((size_t)L.pm * L.pk * 16);
  L.w64 = take((size_t)L.pm * L.pk * 16);
  L.q32 = take((size_t)L.pm * L.pk * 8);
  L.w32 = take((size_t)L.pm * L.pk * 8);
  L.pot = take((size_t)2 * p->n[1] * 8);
  L.fac = take((size_t)nt * S * 4 * nc * nc * cs);
  L.lined = take((size_t)L.lines * 3 * nc * nc * cs);
  L.flag = take(4);
  L.buf = take((size_t)nt * S * nc * cs);
  L.buf2 = p->d >= 2 ? take((size_t)nt * S * nc * cs) : L.buf;
  for (int a = 0; a < 4; a++) {
    L.f64[a] = L.fi64[a] = L.f32[a] = L.fi32[a] = 0;
    L.dpm[a] = L.dpk[a] = 0;
  }
  for (int a = 2; a <= p->d; a++) {
    const int n = p->n[a];
    L.dpm[a] = (n + 63) / 64 * 64;
    L.dpk[a] = (n + 15) / 16 * 16;
    const size_t e = (size_t)L.dpm[a] * L.dpk[a];
    L.f64[a] = take(e * 16);
    L.fi64[a] = take(e * 16);
    L.f32[a] = take(e * 8);
    L.fi32[a] = take(e * 8);
  }
  L.total = off;
  return L;
}

// Y[r][c] = scale * sum_k A[r][k] X[k][c], r < n, c < ncol: a transform along
// one axis of a vector stored with that axis slower than the row of length
// ncol (time: ncol = spatial nodes * nc; transverse axis a: ncol = nodes of
// the faster axes * nc, one matrix per index of the slower axes).  A is
// zero padded to a multiple of 64 rows and 16 columns (row length pk).
// 64 x 64 output tile per workgroup, 4 x 4 per thread (rows ty + 16 i,
// columns tx + 16 j, so that global accesses are coalesced), K in steps of
// 16 through LDS.
// Complex128: the same tile on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
// Real and imaginary parts are staged as separate LDS planes; wavefront w owns
// the 32 x 32 quarter (rows 32 (w >> 1), columns 32 (w & 1)) as 2 x 2 blocks
// of 16 x 16, each a complex product from four real ones
//   Yr += Ar Xr - Ai Xi,  Yi += Ar Xi + Ai Xr.
// Operands: lane l holds A[m = l % 16][k = l / 16] and X[k = l / 16][n = l % 16];
// result register q of lane l is D[l / 16 + 4 q][l % 16] (the FP64 form
// interleaves the rows: measured on gfx950).  Per k step of 4 a wavefront reads
// 8 doubles per lane from LDS for 16 MFMAs (8 flops per byte, against 1 for
// the vector-FMA tile, whose LDS reads bound it).
typedef double d4v_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void tgemm_tile_f64(const double2 *__restrict__ A, int pk,
                                               const double2 *__restrict__ X, double2 *__restrict__ Y, int n,
                                               int64_t ncol, int row0, int64_t col0, double scale) {
  constexpr int LP = 64 + 2;  // plane row length (doubles), padded
  __shared__ double Ar[16][LP], Ai[16][LP], Xr[16][LP], Xi[16][LP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = 32 * (wave >> 1), cb = 32 * (wave & 1);
  const int m = lane & 15, kq = lane >> 4;
  d4v_t accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) accR[i][j] = accI[i][j] = d4v_t{0.0, 0.0, 0.0, 0.0};
  // the next K block of A and X is fetched into registers while the current
  // block's MFMAs run
  double2 pa[4], px[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = threadIdx.x + 256 * q;
      pa[q] = A[(int64_t)(row0 + (e >> 4)) * pk + k0 + (e & 15)];
      const int k = k0 + (e >> 6);
      const int64_t col = col0 + (e & 63);
      px[q] = (k < n && col < ncol) ? X[(int64_t)k * ncol + col] : mk<double2>(0, 0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = threadIdx.x + 256 * q;
      Ar[e & 15][e >> 4] = pa[q].x;
      Ai[e & 15][e >> 4] = pa[q].y;
      Xr[e >> 6][e & 63] = px[q].x;
      Xi[e >> 6][e & 63] = px[q].y;
    }
    __syncthreads();
    if (k0 + 16 < n) fetch(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int kk = ks + kq;
      double ar[2], ai[2], xr[2], xi[2];
#pragma unroll
      for (int i = 0; i < 2; i++) {
        ar[i] = Ar[kk][rb + 16 * i + m];
        ai[i] = Ai[kk][rb + 16 * i + m];
        xr[i] = Xr[kk][cb + 16 * i + m];
        xi[i] = Xi[kk][cb + 16 * i + m];
      }
      // the eight accumulators first take their ar terms, then their ai
      // terms, so that no MFMA waits on the one issued just before it
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], xr[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], xi[j], accI[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], xi[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], xr[j], accI[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int r = row0 + rb + 16 * i + kq + 4 * q;
        const int64_t c = col0 + cb + 16 * j + m;
        if (r < n && c < ncol) Y[(int64_t)r * ncol + c] = mk<double2>(accR[i][j][q] * scale, accI[i][j][q] * scale);
      }
}

template <typename T>
__device__ __forceinline__ void tgemm_tile_fma(const cx<T> *__restrict__ A, int pk, const cx<T> *__restrict__ X,
                                               cx<T> *__restrict__ Y, int n, int64_t ncol, int row0, int64_t col0,
                                               T scale) {
  using C = cx<T>;
  __shared__ C As[16][64];
  __shared__ C Bs[16][64];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  C acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = mk<C>(0, 0);
  for (int k0 = 0; k0 < n; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = threadIdx.x + 256 * q;
      const int r = e >> 4, kk = e & 15;
      As[kk][r] = A[(int64_t)(row0 + r) * pk + k0 + kk];
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = threadIdx.x + 256 * q;
      const int kk = e >> 6, c = e & 63;
      const int k = k0 + kk;
      const int64_t col = col0 + c;
      Bs[kk][c] = (k < n && col < ncol) ? X[(int64_t)k * ncol + col] : mk<C>(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk++) {
      C a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int r = row0 + ty + 16 * i;
    if (r >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t c = col0 + tx + 16 * j;
      if (c < ncol) Y[(int64_t)r * ncol + c] = mk<C>(acc[i][j].x * scale, acc[i][j].y * scale);
    }
  }
}

// complex128 on the matrix cores, complex64 with vector FMAs
template <typename T>
__device__ __forceinline__ void tgemm_tile(const cx<T> *__restrict__ A, int pk, const cx<T> *__restrict__ X,
                                  cx<T> *__restrict__ Y, int n, int64_t ncol, int row0, int64_t col0,
                                  T scale) {
  if constexpr (sizeof(T) == 8)
    tgemm_tile_f64(A, pk, X, Y, n, ncol, row0, col0, scale);
  else
    tgemm_tile_fma<T>(A, pk, X, Y, n, ncol, row0, col0, scale);
}

// grid: (column tiles, row tiles, batches); batch b works on X + b n ncol
template <typename T>
__global__ __launch_bounds__(256) void tgemm(const cx<T> *__restrict__ A, int pk,
                                             const cx<T> *__restrict__ X, cx<T> *__restrict__ Y,
                                             int n, int64_t ncol, T scale) {
  const int64_t boff = (int64_t)blockIdx.z * n * ncol;
  tgemm_tile<T>(A, pk, X + boff, Y + boff, n, ncol, blockIdx.y * 64, (int64_t)blockIdx.x * 64, scale);
}

template <int NC>
__device__ inline void blk_axpy(double2 *out, const double2 *a, double s, const double2 *b) {
#pragma unroll
  for (int q = 0; q < NC * NC; q++) out[q] = mk<double2>(a[q].x + s * b[q].x, a[q].y + s * b[q].y);
}

template <int NC>
__device__ inline bool blk_finite(const double2 *a) {
  bool ok = true;
#pragma unroll
  for (int q = 0; q < NC * NC; q++) ok = ok && isfinite(a[q].x) && isfinite(a[q].y);
  return ok;
}

// Factors per node, layout [i_1][slot][q][line] (slot 0 G_i, 1 K_i = G_i L_i,
// 2 E_i, 3 H_i), per line [slot][q][line] (slot 0 L_{n-1}, 1 U_{n-1} (the
// corner coupling to node 0), 2 S^{-1}).  One thread per line; the
// forward sweep writes F_i into the H slot, the backward sweep replaces it.
template <typename T, int NC, int DS>
__device__ __forceinline__ void line_setup_one(const SpecGeom &G, const double2 *__restrict__ tw,
                                               const double2 *__restrict__ lam,
                                               const double *__restrict__ pot, cx<T> *__restrict__ fac,
                                               cx<T> *__restrict__ lined, int64_t lines,
                                               int *__restrict__ flag, int64_t l) {
  constexpr int B = NC * NC;
  const int n1 = G.n[1];
  const int64_t nperp = G.S / n1;
  const int tq = (int)(l / nperp);
  int64_t rem = l - (int64_t)tq * nperp;
  double mu[DS + 1], sn[DS + 1];
  double mperp = 1.0;
#pragma unroll
  for (int a = 2; a <= DS; a++) {
    const int k = (int)(rem % G.n[a]);
    rem /= G.n[a];
    const double2 w = tw[G.tw_off[a] + k];  // exp(-i th)
    mu[a] = G.h[a] * (2.0 + w.x) / 3.0;
    sn[a] = -w.y;
    mperp *= mu[a];
  }
  const double2 lm = lam[tq];
  const double h1 = G.h[1];
  double2 AL[B], AD[B], AU[B], CP[B];
#pragma unroll
  for (int q = 0; q < B; q++) {
    const int i = q / NC, j = q % NC;
    const double2 g0 = G.g[0][q], g1 = G.g[1][q];
    // i lambda mu g0
    const double2 il = mk<double2>(-lm.y * mperp, lm.x * mperp);
    double2 cm = cmul(il, g0);
    if (i == j) cm.x -= G.m * mperp;
#pragma unroll
    for (int a = 2; a <= DS; a++) {
      double other = 1.0;
#pragma unroll
      for (int b = 2; b <= DS; b++)
        if (b != a) other *= mu[b];
      // i g_a (i sin th_a) other = -g_a sin th_a other
      cm.x -= G.g[a][q].x * sn[a] * other;
      cm.y -= G.g[a][q].y * sn[a] * other;
    }
    const double2 cd = mk<double2>(-g1.y * mperp, g1.x * mperp);  // i mu g1
    AL[q] = mk<double2>(h1 / 6.0 * cm.x - 0.5 * cd.x, h1 / 6.0 * cm.y - 0.5 * cd.y);
    AU[q] = mk<double2>(h1 / 6.0 * cm.x + 0.5 * cd.x, h1 / 6.0 * cm.y + 0.5 * cd.y);
    AD[q] = mk<double2>(2.0 * h1 / 3.0 * cm.x, 2.0 * h1 / 3.0 * cm.y);
    CP[q] = mk<double2>(mperp * g0.x, mperp * g0.y);
  }
  const double *pdiag = pot, *poff = pot + n1;
  auto fidx = [&](int i, int slot, int q) { return ((int64_t)i * 4 * B + slot * B + q) * lines + l; };
  double2 E[B], F[B], Li[B], Di[B], Ui[B], tmp[B], Gi[B], col[B];
#pragma unroll
  for (int q = 0; q < B; q++) E[q] = F[q] = mk<double2>(0, 0);
  bool ok = true;
  for (int i = 0; i < n1 - 1; i++) {
    blk_axpy<NC>(Li, AL, -poff[i == 0 ? n1 - 1 : i - 1], CP);
    blk_axpy<NC>(Di, AD, -pdiag[i], CP);
    blk_axpy<NC>(Ui, AU, -poff[i], CP);
    // pivot D_i - L_i E_{i-1}
    matmul_nc<NC>(Li, E, tmp);
#pragma unroll
    for (int q = 0; q < B; q++) tmp[q] = csub(Di[q], tmp[q]);
    inverse_nc<NC>(tmp, Gi);
    ok = ok && blk_finite<NC>(Gi);
    // border column: corner L_0 in row 0, U_{n-2} in row n-2, minus L_i F_{i-1}
    matmul_nc<NC>(Li, F, tmp);
#pragma unroll
    for (int q = 0; q < B; q++) {
      double2 c = i > 0 ? mk<double2>(-tmp[q].x, -tmp[q].y) : Li[q];
      if (i == n1 - 2) c = cadd(c, Ui[q]);
      col[q] = c;
    }
    matmul_nc<NC>(Gi, col, F);
    if (i < n1 - 2) {
      matmul_nc<NC>(Gi, Ui, E);
    } else {
#pragma unroll
      for (int q = 0; q < B; q++) E[q] = mk<double2>(0, 0);
    }
    if (i > 0) {
      matmul_nc<NC>(Gi, Li, tmp);
    } else {
#pragma unroll
      for (int q = 0; q < B; q++) tmp[q] = mk<double2>(0, 0);
    }
#pragma unroll
    for (int q = 0; q < B; q++) {
      fac[fidx(i, 0, q)] = mk<cx<T>>((T)Gi[q].x, (T)Gi[q].y);
      fac[fidx(i, 1, q)] = mk<cx<T>>((T)tmp[q].x, (T)tmp[q].y);
      fac[fidx(i, 2, q)] = mk<cx<T>>((T)E[q].x, (T)E[q].y);
      fac[fidx(i, 3, q)] = mk<cx<T>>((T)F[q].x, (T)F[q].y);
    }
  }
  // backward: H_{n-2} = -F_{n-2}, H_i = -E_i H_{i+1} - F_i (E_i and F_i are
  // read back at the storage precision; H is carried in FP64)
  double2 H[B], Hl[B];
#pragma unroll
  for (int q = 0; q < B; q++) {
    H[q] = mk<double2>(-F[q].x, -F[q].y);
    Hl[q] = H[q];
    fac[fidx(n1 - 2, 3, q)] = mk<cx<T>>((T)H[q].x, (T)H[q].y);
  }
  for (int i = n1 - 3; i >= 0; i--) {
#pragma unroll
    for (int q = 0; q < B; q++) {
      const cx<T> e = fac[fidx(i, 2, q)], f = fac[fidx(i, 3, q)];
      E[q] = mk<double2>((double)e.x, (double)e.y);
      F[q] = mk<double2>((double)f.x, (double)f.y);
    }
    matmul_nc<NC>(E, H, tmp);
#pragma unroll
    for (int q = 0; q < B; q++) {
      H[q] = mk<double2>(-tmp[q].x - F[q].x, -tmp[q].y - F[q].y);
      fac[fidx(i, 3, q)] = mk<cx<T>>((T)H[q].x, (T)H[q].y);
    }
  }
  // Schur complement of the last node: D_{n-1} + L_{n-1} H_{n-2} + U_{n-1} H_0
  blk_axpy<NC>(Li, AL, -poff[n1 - 2], CP);
  blk_axpy<NC>(Di, AD, -pdiag[n1 - 1], CP);
  blk_axpy<NC>(Ui, AU, -poff[n1 - 1], CP);
  matmul_nc<NC>(Li, Hl, tmp);
  matmul_nc<NC>(Ui, H, col);
#pragma unroll
  for (int q = 0; q < B; q++) tmp[q] = cadd(Di[q], cadd(tmp[q], col[q]));
  inverse_nc<NC>(tmp, Gi);
  ok = ok && blk_finite<NC>(Gi);
#pragma unroll
  for (int q = 0; q < B; q++) {
    lined[(0 * B + q) * lines + l] = mk<cx<T>>((T)Li[q].x, (T)Li[q].y);
    lined[(1 * B + q) * lines + l] = mk<cx<T>>((T)Ui[q].x, (T)Ui[q].y);
    lined[(2 * B + q) * lines + l] = mk<cx<T>>((T)Gi[q].x, (T)Gi[q].y);
  }
  if (!ok) atomicAdd(flag, 1);
}

template <typename T, int NC, int DS>
__global__ __launch_bounds__(64) void line_setup(SpecGeom G, const double2 *__restrict__ tw,
                                                 const double2 *__restrict__ lam,
                                                 const double *__restrict__ pot,
                                                 cx<T> *__restrict__ fac, cx<T> *__restrict__ lined,
                                                 int64_t lines, int *__restrict__ flag) {
  const int64_t l = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (l < lines) line_setup_one<T, NC, DS>(G, tw, lam, pot, fac, lined, lines, flag, l);
}

// In-place periodic block-tridiagonal solve along x, one thread per line
// (line l holds nodes l * n1 .. l * n1 + n1 - 1, nc components each).
template <typename T, int NC>
__device__ __forceinline__ void blk_load(const cx<T> *__restrict__ fac, int64_t base, int64_t lines,
                                         cx<T> (&m)[NC * NC]) {
#pragma unroll
  for (int q = 0; q < NC * NC; q++) m[q] = fac[base + (int64_t)q * lines];
}

template <typename T, int NC>
__device__ __forceinline__ void blk_apply(const cx<T> (&m)[NC * NC], const cx<T> *v, cx<T> *out, bool accum,
                                          bool neg) {
#pragma unroll
  for (int i = 0; i < NC; i++) {
    cx<T> s = accum ? out[i] : mk<cx<T>>(0, 0);
#pragma unroll
    for (int j = 0; j < NC; j++) s = neg ? cfms(s, m[i * NC + j], v[j]) : cfma(s, m[i * NC + j], v[j]);
    out[i] = s;
  }
}

// In-place periodic block-tridiagonal solve along x for line l (nodes
// l * n1 .. l * n1 + n1 - 1, nc components each), one thread per line with
// no cooperation: each sweep loads the next node's factors and values one
// step ahead, so the loads overlap the dependent arithmetic of the current
// node.  Used when there are too few lines for the LDS-staged workgroup
// version to fill the chip.
template <typename T, int NC>
__device__ __forceinline__ void line_solve_thread(const cx<T> *__restrict__ fac, const cx<T> *__restrict__ lined,
                                               cx<T> *__restrict__ X, int n1, int64_t lines, int64_t l) {
  constexpr int B = NC * NC;
  using C = cx<T>;
  C *x = X + l * n1 * NC;
  auto fb = [&](int i, int slot) { return ((int64_t)i * 4 * B + slot * B) * lines + l; };
  C y[NC], t[NC], v[NC], vn[NC];
  C Gm[B], Km[B], Gn[B], Kn[B];
#pragma unroll
  for (int c = 0; c < NC; c++) y[c] = vn[c] = mk<C>(0, 0);
#pragma unroll
  for (int q = 0; q < B; q++) Gn[q] = Kn[q] = mk<C>(0, 0);
  // forward: y_i = G_i v_i - K_i y_{i-1}
  blk_load<T, NC>(fac, fb(0, 0), lines, Gm);
  blk_load<T, NC>(fac, fb(0, 1), lines, Km);
#pragma unroll
  for (int c = 0; c < NC; c++) v[c] = x[c];
  for (int i = 0; i < n1 - 1; i++) {
    if (i + 1 < n1 - 1) {
      blk_load<T, NC>(fac, fb(i + 1, 0), lines, Gn);
      blk_load<T, NC>(fac, fb(i + 1, 1), lines, Kn);
#pragma unroll
      for (int c = 0; c < NC; c++) vn[c] = x[(i + 1) * NC + c];
    }
    blk_apply<T, NC>(Gm, v, t, false, false);
    blk_apply<T, NC>(Km, y, t, true, true);
#pragma unroll
    for (int c = 0; c < NC; c++) {
      y[c] = t[c];
      x[i * NC + c] = t[c];
    }
#pragma unroll
    for (int q = 0; q < B; q++) {
      Gm[q] = Gn[q];
      Km[q] = Kn[q];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = vn[c];
  }
  // backward: a_i = y_i - E_i a_{i+1}
  C alast[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) alast[c] = y[c];
  if (n1 >= 3) {
    blk_load<T, NC>(fac, fb(n1 - 3, 2), lines, Gm);
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = x[(n1 - 3) * NC + c];
  }
  for (int i = n1 - 3; i >= 0; i--) {
    if (i > 0) {
      blk_load<T, NC>(fac, fb(i - 1, 2), lines, Gn);
#pragma unroll
      for (int c = 0; c < NC; c++) vn[c] = x[(i - 1) * NC + c];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) t[c] = v[c];
    blk_apply<T, NC>(Gm, y, t, true, true);
#pragma unroll
    for (int c = 0; c < NC; c++) {
      y[c] = t[c];
      x[i * NC + c] = t[c];
    }
#pragma unroll
    for (int q = 0; q < B; q++) Gm[q] = Gn[q];
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = vn[c];
  }
  // last node: S^{-1} (v_{n-1} - L_{n-1} a_{n-2} - U_{n-1} a_0)
#pragma unroll
  for (int c = 0; c < NC; c++) t[c] = x[(n1 - 1) * NC + c];
  blk_load<T, NC>(lined, 0 * B * lines + l, lines, Gm);
  blk_apply<T, NC>(Gm, alast, t, true, true);
  blk_load<T, NC>(lined, 1 * B * lines + l, lines, Gm);
  blk_apply<T, NC>(Gm, y, t, true, true);
  C xl[NC];
  blk_load<T, NC>(lined, 2 * B * lines + l, lines, Gm);
  blk_apply<T, NC>(Gm, t, xl, false, false);
#pragma unroll
  for (int c = 0; c < NC; c++) x[(n1 - 1) * NC + c] = xl[c];
  // x_i = a_i + H_i x_{n-1}
  blk_load<T, NC>(fac, fb(0, 3), lines, Gm);
#pragma unroll
  for (int c = 0; c < NC; c++) v[c] = x[c];
  for (int i = 0; i < n1 - 1; i++) {
    if (i + 1 < n1 - 1) {
      blk_load<T, NC>(fac, fb(i + 1, 3), lines, Gn);
#pragma unroll
      for (int c = 0; c < NC; c++) vn[c] = x[(i + 1) * NC + c];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) t[c] = v[c];
    blk_apply<T, NC>(Gm, xl, t, true, false);
#pragma unroll
    for (int c = 0; c < NC; c++) x[i * NC + c] = t[c];
#pragma unroll
    for (int q = 0; q < B; q++) Gm[q] = Gn[q];
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = vn[c];
  }
}

// The same solve for 2 x 2 blocks with the node loads issued PF nodes at a
// time: every sweep loads the factors and values of the next PF nodes before
// their dependent arithmetic, so PF memory latencies overlap instead of one
// (the kernel runs one thread per line and about one wavefront per compute
// unit, so latency, not bandwidth, is what bounds it).  The correction sweep
// has no dependency between nodes at all.
template <typename T, int PF>
__device__ __forceinline__ void line_solve_thread2(const cx<T> *__restrict__ fac, const cx<T> *__restrict__ lined,
                                                cx<T> *__restrict__ X, int n1, int64_t lines, int64_t l) {
  constexpr int NC = 2, B = NC * NC;
  using C = cx<T>;
  C *x = X + l * n1 * NC;
  auto fb = [&](int i, int slot) { return ((int64_t)i * 4 * B + slot * B) * lines + l; };
  C y[NC], t[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) y[c] = mk<C>(0, 0);
  // forward: y_i = G_i v_i - K_i y_{i-1}
  for (int i0 = 0; i0 < n1 - 1; i0 += PF) {
    C Gb[PF][B], Kb[PF][B], vb[PF][NC];
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int i = i0 + u;
      if (i < n1 - 1) {
        blk_load<T, NC>(fac, fb(i, 0), lines, Gb[u]);
        blk_load<T, NC>(fac, fb(i, 1), lines, Kb[u]);
#pragma unroll
        for (int c = 0; c < NC; c++) vb[u][c] = x[i * NC + c];
      }
    }
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int i = i0 + u;
      if (i < n1 - 1) {
        blk_apply<T, NC>(Gb[u], vb[u], t, false, false);
        blk_apply<T, NC>(Kb[u], y, t, true, true);
#pragma unroll
        for (int c = 0; c < NC; c++) {
          y[c] = t[c];
          x[i * NC + c] = t[c];
        }
      }
    }
  }
  // backward: a_i = y_i - E_i a_{i+1}, from a_{n-2} = y_{n-2}
  C alast[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) alast[c] = y[c];
  for (int i0 = n1 - 3; i0 >= 0; i0 -= PF) {
    C Eb[PF][B], vb[PF][NC];
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int i = i0 - u;
      if (i >= 0) {
        blk_load<T, NC>(fac, fb(i, 2), lines, Eb[u]);
#pragma unroll
        for (int c = 0; c < NC; c++) vb[u][c] = x[i * NC + c];
      }
    }
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int i = i0 - u;
      if (i >= 0) {
#pragma unroll
        for (int c = 0; c < NC; c++) t[c] = vb[u][c];
        blk_apply<T, NC>(Eb[u], y, t, true, true);
#pragma unroll
        for (int c = 0; c < NC; c++) {
          y[c] = t[c];
          x[i * NC + c] = t[c];
        }
      }
    }
  }
  // last node: S^{-1} (v_{n-1} - L_{n-1} a_{n-2} - U_{n-1} a_0)
  C Mq[B];
#pragma unroll
  for (int c = 0; c < NC; c++) t[c] = x[(n1 - 1) * NC + c];
  blk_load<T, NC>(lined, 0 * B * lines + l, lines, Mq);
  blk_apply<T, NC>(Mq, alast, t, true, true);
  blk_load<T, NC>(lined, 1 * B * lines + l, lines, Mq);
  blk_apply<T, NC>(Mq, y, t, true, true);
  C xl[NC];
  blk_load<T, NC>(lined, 2 * B * lines + l, lines, Mq);
  blk_apply<T, NC>(Mq, t, xl, false, false);
#pragma unroll
  for (int c = 0; c < NC; c++) x[(n1 - 1) * NC + c] = xl[c];
  // x_i = a_i + H_i x_{n-1}
  for (int i0 = 0; i0 < n1 - 1; i0 += PF) {
    C Hb[PF][B], vb[PF][NC];
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int i = i0 + u;
      if (i < n1 - 1) {
        blk_load<T, NC>(fac, fb(i, 3), lines, Hb[u]);
#pragma unroll
        for (int c = 0; c < NC; c++) vb[u][c] = x[i * NC + c];
      }
    }
#pragma unroll
    for (int u = 0; u < PF; u++) {
      const int i = i0 + u;
      if (i < n1 - 1) {
        blk_apply<T, NC>(Hb[u], xl, vb[u], true, false);
#pragma unroll
        for (int c = 0; c < NC; c++) x[i * NC + c] = vb[u][c];
      }
    }
  }
}

// In-place periodic block-tridiagonal solve along x for the 64 lines
// l0 .. l0 + 63 of one workgroup (line l holds nodes l * n1 .. l * n1 + n1 - 1,
// nc components each); thread t owns line l0 + t.  The line values move
// through LDS in chunks of CH nodes: the workgroup loads a chunk of all its
// lines cooperatively (contiguous 16-byte pieces, coalesced), each thread
// sweeps its own line inside the chunk, and the chunk is stored back the same
// way.  The factors are laid out [node][entry][line], so their per-thread
// loads are coalesced already; they are fetched one node ahead.
template <typename T, int NC, int CH>
__device__ __forceinline__ void line_solve_wg(const cx<T> *__restrict__ fac, const cx<T> *__restrict__ lined,
                                              cx<T> *__restrict__ X, int n1, int64_t lines, int64_t l0) {
  constexpr int B = NC * NC, CL = CH * NC, RL = CL + 1;  // padded LDS row
  using C = cx<T>;
  __shared__ C sh[64][RL];
  const int t = threadIdx.x;
  const int64_t l = l0 + t;
  const bool own = l < lines;
  const int64_t lc = own ? l : l0;  // a valid line for the factor addresses of idle threads
  auto fb = [&](int i, int slot) { return ((int64_t)i * 4 * B + slot * B) * lines + lc; };
  auto load_chunk = [&](int i0) {
#pragma unroll 4
    for (int k = 0; k < CL; k++) {
      const int e = t + 64 * k, ln = e / CL, r = e - ln * CL;
      const bool ok = l0 + ln < lines && i0 + r / NC < n1;
      sh[ln][r] = ok ? X[(l0 + ln) * n1 * NC + (int64_t)i0 * NC + r] : mk<C>(0, 0);
    }
    __syncthreads();
  };
  auto store_chunk = [&](int i0) {
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < CL; k++) {
      const int e = t + 64 * k, ln = e / CL, r = e - ln * CL;
      if (l0 + ln < lines && i0 + r / NC < n1) X[(l0 + ln) * n1 * NC + (int64_t)i0 * NC + r] = sh[ln][r];
    }
    __syncthreads();
  };
  C y[NC], tv[NC], Gm[B], Km[B], Gn[B], Kn[B];
#pragma unroll
  for (int c = 0; c < NC; c++) y[c] = mk<C>(0, 0);
#pragma unroll
  for (int q = 0; q < B; q++) Gn[q] = Kn[q] = mk<C>(0, 0);
  // forward: y_i = G_i v_i - K_i y_{i-1}, nodes 0 .. n1-2
  blk_load<T, NC>(fac, fb(0, 0), lines, Gm);
  blk_load<T, NC>(fac, fb(0, 1), lines, Km);
  for (int i0 = 0; i0 < n1 - 1; i0 += CH) {
    load_chunk(i0);
    const int ie = min(i0 + CH, n1 - 1);
    for (int i = i0; i < ie; i++) {
      if (i + 1 < n1 - 1) {
        blk_load<T, NC>(fac, fb(i + 1, 0), lines, Gn);
        blk_load<T, NC>(fac, fb(i + 1, 1), lines, Kn);
      }
      C v[NC];
#pragma unroll
      for (int c = 0; c < NC; c++) v[c] = sh[t][(i - i0) * NC + c];
      blk_apply<T, NC>(Gm, v, tv, false, false);
      blk_apply<T, NC>(Km, y, tv, true, true);
#pragma unroll
      for (int c = 0; c < NC; c++) {
        y[c] = tv[c];
        sh[t][(i - i0) * NC + c] = tv[c];
      }
#pragma unroll
      for (int q = 0; q < B; q++) {
        Gm[q] = Gn[q];
        Km[q] = Kn[q];
      }
    }
    store_chunk(i0);
  }
  // backward: a_i = y_i - E_i a_{i+1}, nodes n1-3 .. 0
  C alast[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) alast[c] = y[c];
  blk_load<T, NC>(fac, fb(n1 - 3, 2), lines, Gm);
  for (int i0 = ((n1 - 3) / CH) * CH; i0 >= 0; i0 -= CH) {
    load_chunk(i0);
    for (int i = min(i0 + CH - 1, n1 - 3); i >= i0; i--) {
      if (i > 0) blk_load<T, NC>(fac, fb(i - 1, 2), lines, Gn);
#pragma unroll
      for (int c = 0; c < NC; c++) tv[c] = sh[t][(i - i0) * NC + c];
      blk_apply<T, NC>(Gm, y, tv, true, true);
#pragma unroll
      for (int c = 0; c < NC; c++) {
        y[c] = tv[c];
        sh[t][(i - i0) * NC + c] = tv[c];
      }
#pragma unroll
      for (int q = 0; q < B; q++) Gm[q] = Gn[q];
    }
    store_chunk(i0);
  }
  // last node: S^{-1} (v_{n-1} - L_{n-1} a_{n-2} - U_{n-1} a_0)
  C xl[NC];
  {
    const int64_t ll = lc - l0;  // 0 for idle threads; their results are never stored
    (void)ll;
#pragma unroll
    for (int c = 0; c < NC; c++) tv[c] = X[lc * n1 * NC + (int64_t)(n1 - 1) * NC + c];
    blk_load<T, NC>(lined, 0 * B * lines + lc, lines, Gm);
    blk_apply<T, NC>(Gm, alast, tv, true, true);
    blk_load<T, NC>(lined, 1 * B * lines + lc, lines, Gm);
    blk_apply<T, NC>(Gm, y, tv, true, true);
    blk_load<T, NC>(lined, 2 * B * lines + lc, lines, Gm);
    blk_apply<T, NC>(Gm, tv, xl, false, false);
  }
  __syncthreads();  // every thread has read v_{n-1} of its line before any is overwritten
  if (own) {
#pragma unroll
    for (int c = 0; c < NC; c++) X[l * n1 * NC + (int64_t)(n1 - 1) * NC + c] = xl[c];
  }
  __syncthreads();
  // x_i = a_i + H_i x_{n-1}, nodes 0 .. n1-2
  blk_load<T, NC>(fac, fb(0, 3), lines, Gm);
  for (int i0 = 0; i0 < n1 - 1; i0 += CH) {
    load_chunk(i0);
    const int ie = min(i0 + CH, n1 - 1);
    for (int i = i0; i < ie; i++) {
      if (i + 1 < n1 - 1) blk_load<T, NC>(fac, fb(i + 1, 3), lines, Gn);
#pragma unroll
      for (int c = 0; c < NC; c++) tv[c] = sh[t][(i - i0) * NC + c];
      blk_apply<T, NC>(Gm, xl, tv, true, false);
#pragma unroll
      for (int c = 0; c < NC; c++) sh[t][(i - i0) * NC + c] = tv[c];
#pragma unroll
      for (int q = 0; q < B; q++) Gm[q] = Gn[q];
    }
    store_chunk(i0);
  }
}

// chunk length of the LDS-staged line solve (nodes)
constexpr int kLineChunk = 8;
constexpr int kLinePF = 8;  // nodes per load round of the one-thread-per-line solve (2 x 2 blocks)

template <typename T, int NC>
__global__ __launch_bounds__(64) void line_solve(const cx<T> *__restrict__ fac,
                                                 const cx<T> *__restrict__ lined,
                                                 cx<T> *__restrict__ X, int n1, int64_t lines) {
  line_solve_wg<T, NC, kLineChunk>(fac, lined, X, n1, lines, (int64_t)blockIdx.x * 64);
}

template <typename T, int NC>
__global__ __launch_bounds__(64) void line_solve_pt(const cx<T> *__restrict__ fac,
                                                    const cx<T> *__restrict__ lined,
                                                    cx<T> *__restrict__ X, int n1, int64_t lines) {
  const int64_t l = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (l >= lines) return;
  if constexpr (NC == 2) line_solve_thread2<T, kLinePF>(fac, lined, X, n1, lines, l);
  else line_solve_thread<T, NC>(fac, lined, X, n1, lines, l);
}

// below this many lines a single system's solve runs one thread per line
constexpr int64_t kLineStagedMin = 65536;

static __global__ void zero_i32_flag(int *f) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *f = 0;
}

}  // namespace dst
