// spmv.hpp -- block-CSR SpMV kernels (y = alpha A x and r = b - A x).
//
// The product inside GMRES (Sec. 2.2).  Work split: G consecutive lanes own
// one block row.  The row's values are contiguous ([nnzb][nc][nc]), so the
// group walks them in 16-byte chunks: lane l always reads chunk l of each
// G-chunk slice, which keeps the wavefront's loads fully coalesced and fixes
// the output component i of every lane.  A chunk is one complex128 entry, or
// two adjacent complex64 entries of the same block row (16 bytes either way);
// the x operand of a chunk is the matching 16 bytes of the column node.
// complex128 values are streamed with nontemporal loads so that x stays in
// cache; for complex64 plain loads measured faster (65 % vs 57 % of HBM peak
// at 2+1D 128^3).
// Partial sums are combined with xor shuffles over the lane bits that do not
// encode i.  Tiles of rows are assigned so that each XCD gets a contiguous
// share of rows (x reuse in that XCD's L2).
#pragma once

#include "common.hpp"

namespace dst {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));

// 16-byte chunk: one complex128 or two complex64 values (clang vector types,
// so the nontemporal load builtin accepts them)
template <typename T> struct chunk_of;
template <> struct chunk_of<double> { using type = dv2; static constexpr int J = 1; };
template <> struct chunk_of<float> { using type = fv4; static constexpr int J = 2; };

template <typename T>
__device__ inline cx<T> chunk_mac(cx<T> acc, typename chunk_of<T>::type v, typename chunk_of<T>::type x);
template <>
__device__ inline double2 chunk_mac<double>(double2 acc, dv2 v, dv2 x) {
  return cfma(acc, mk<double2>(v.x, v.y), mk<double2>(x.x, x.y));
}
template <>
__device__ inline float2 chunk_mac<float>(float2 acc, fv4 v, fv4 x) {
  acc = cfma(acc, mk<float2>(v.x, v.y), mk<float2>(x.x, x.y));
  return cfma(acc, mk<float2>(v.z, v.w), mk<float2>(x.z, x.w));
}

// Rows [tile * 256/G, (tile + 1) * 256/G) of one operator, one workgroup.
template <typename T, int NC, int G, bool RESID>
__device__ __forceinline__ void spmv_tile(int64_t tile, int64_t nrows, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ ci, const cx<T> *__restrict__ val,
                                 const cx<T> *__restrict__ x, const cx<T> *__restrict__ bvec,
                                 cx<T> *__restrict__ y, T alpha) {
  using Ch = typename chunk_of<T>::type;
  constexpr int J = chunk_of<T>::J;
  constexpr int IB = NC / J;          // chunks per block row
  constexpr int CPB = NC * NC / J;    // chunks per block
  constexpr int BPI = G / CPB;        // blocks per group slice
  constexpr int RPW = 256 / G;        // rows per workgroup
  constexpr int IMASK = (NC - 1) * IB;
  static_assert(G % CPB == 0 && G <= 64, "group must hold whole blocks");
  const int lane = threadIdx.x % G;
  const int64_t row = tile * RPW + threadIdx.x / G;
  const int i = (lane / IB) % NC;
  const int jc = lane % IB;
  const int bofs = lane / CPB;
  // a row holds at most 3^(d+1) blocks: 27 (2x2 blocks, d <= 2) or 81 (4x4, d = 3)
  constexpr int MAXB = NC == 2 ? 27 : 81;
  constexpr int MAXIT = (MAXB + BPI - 1) / BPI;
  constexpr int UNR = MAXIT < 8 ? MAXIT : 8;
  cx<T> acc = mk<cx<T>>(0, 0);
  if (row < nrows) {
    const int rs = rp[row], re = rp[row + 1];
    const Ch *vbase = reinterpret_cast<const Ch *>(val + i * NC + jc * J);
    // batches of UNR slices: all value, index and x loads of a batch are in
    // flight before its first multiply
    for (int b0 = rs + bofs; b0 < re; b0 += UNR * BPI) {
      Ch v[UNR], xv[UNR];
      int c[UNR];
#pragma unroll
      for (int it = 0; it < UNR; it++) {
        const int b = b0 + it * BPI;
        if (b < re) {
          if constexpr (sizeof(T) == 8) v[it] = __builtin_nontemporal_load(vbase + (int64_t)b * (NC * NC / J));
          else v[it] = vbase[(int64_t)b * (NC * NC / J)];
          c[it] = ci[b];
        }
      }
#pragma unroll
      for (int it = 0; it < UNR; it++) {
        const int b = b0 + it * BPI;
        if (b < re) xv[it] = *reinterpret_cast<const Ch *>(x + (int64_t)c[it] * NC + jc * J);
      }
#pragma unroll
      for (int it = 0; it < UNR; it++) {
        const int b = b0 + it * BPI;
        if (b < re) acc = chunk_mac<T>(acc, v[it], xv[it]);
      }
    }
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    if (off & IMASK) continue;
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
  }
  if (row < nrows && lane == i * IB) {
    const int64_t o = row * NC + i;
    if (RESID) {
      cx<T> bb = bvec[o];
      y[o] = mk<cx<T>>(bb.x - acc.x, bb.y - acc.y);
    } else {
      y[o] = mk<cx<T>>(alpha * acc.x, alpha * acc.y);
    }
  }
}

// Block-row structure of the assembled operator, used to address blocks and
// columns without reading row_ptr / col_idx.  A row (time node tau = 1..n_t,
// spatial node with coordinates i_a) couples to the 3^d spatial neighbours
// (periodic) in each of the time nodes tau-1 (if tau >= 2), tau, tau+1 (if
// tau <= n_t - 1); its blocks are stored in ascending column order.
struct Stencil {
  int d, nt;
  int n[4];    // n[1..d] spatial nodes per axis
  int64_t S;   // spatial nodes
  int P;       // 3^d
};

inline Stencil make_stencil(const dirac_st_problem *p) {
  Stencil g{};
  g.d = p->d;
  g.nt = p->n[0];
  g.S = 1;
  g.P = 1;
  for (int a = 1; a <= 3; a++) g.n[a] = a <= p->d ? p->n[a] : 1;
  for (int a = 1; a <= p->d; a++) {
    g.S *= p->n[a];
    g.P *= 3;
  }
  return g;
}

// coordinate of sorted neighbour k (0, 1, 2) of i on a periodic axis of n >= 3
// nodes: the set {i-1, i, i+1} mod n in ascending order
__device__ __forceinline__ int nb_coord(int i, int n, int k) {
  if (i == 0) return k == 2 ? n - 1 : k;
  if (i == n - 1) return k == 0 ? 0 : n - 3 + k;
  return i - 1 + k;
}

// first block and block count of a row
template <int DS>
__device__ __forceinline__ void st_row(const Stencil &g, int64_t row, int64_t &rs, int &nb) {
  const int tau = (int)(row / g.S) + 1;
  const int64_t s = row - (int64_t)(tau - 1) * g.S;
  const int P = g.P;
  if (g.nt == 1) {
    rs = row * P;
    nb = P;
    return;
  }
  const int mid = 3 * P, edge = 2 * P;
  if (tau == 1) {
    rs = s * edge;
  } else {
    rs = g.S * edge + (int64_t)(tau - 2) * g.S * mid + s * (tau == g.nt ? edge : mid);
  }
  nb = (tau == 1 || tau == g.nt) ? edge : mid;
}

// spmv_tile without index traffic: same work split and value stream as
// spmv_tile, block range and columns computed from the stencil
template <typename T, int NC, int DS, int G, bool RESID>
__device__ __forceinline__ void spmv_tile_st(int64_t tile, int64_t nrows, const Stencil &g,
                                             const cx<T> *__restrict__ val, const cx<T> *__restrict__ x,
                                             const cx<T> *__restrict__ bvec, cx<T> *__restrict__ y, T alpha) {
  using Ch = typename chunk_of<T>::type;
  constexpr int J = chunk_of<T>::J;
  constexpr int IB = NC / J;
  constexpr int CPB = NC * NC / J;
  constexpr int BPI = G / CPB;
  constexpr int RPW = 256 / G;
  constexpr int IMASK = (NC - 1) * IB;
  static_assert(G % CPB == 0 && G <= 64, "group must hold whole blocks");
  const int lane = threadIdx.x % G;
  const int64_t row = tile * RPW + threadIdx.x / G;
  const int i = (lane / IB) % NC;
  const int jc = lane % IB;
  const int bofs = lane / CPB;
  constexpr int MAXB = NC == 2 ? 27 : 81;
  constexpr int MAXIT = (MAXB + BPI - 1) / BPI;
  constexpr int UNR = MAXIT < 8 ? MAXIT : 8;
  cx<T> acc = mk<cx<T>>(0, 0);
  if (row < nrows) {
    int64_t rs;
    int nb;
    st_row<DS>(g, row, rs, nb);
    const int tau = (int)(row / g.S) + 1;
    int64_t sr = row - (int64_t)(tau - 1) * g.S;
    // per axis: element offsets (in x, nc-blocks) of the three sorted
    // neighbours; per block only digit extraction by constants and selects
    constexpr int P = DS == 1 ? 3 : DS == 2 ? 9 : 27;
    int off[DS + 1][3];
    int stride = 1;
#pragma unroll
    for (int a = 1; a <= DS; a++) {
      const int n = g.n[a];
      const int ia = (int)(sr % n);
      sr /= n;
#pragma unroll
      for (int k = 0; k < 3; k++) off[a][k] = nb_coord(ia, n, k) * stride;
      stride *= n;
    }
    const int64_t tbase = (int64_t)((tau >= 2 ? tau - 1 : tau) - 1) * g.S;
    const Ch *vbase = reinterpret_cast<const Ch *>(val + rs * NC * NC + i * NC + jc * J);
    for (int b0 = bofs; b0 < nb; b0 += UNR * BPI) {
      Ch v[UNR], xv[UNR];
#pragma unroll
      for (int it = 0; it < UNR; it++) {
        const int b = b0 + it * BPI;
        if (b < nb) {
          if constexpr (sizeof(T) == 8) v[it] = __builtin_nontemporal_load(vbase + (int64_t)b * (NC * NC / J));
          else v[it] = vbase[(int64_t)b * (NC * NC / J)];
          const int kt = b / P;
          int rem = b - kt * P;
          int64_t c = tbase + (int64_t)kt * g.S;
#pragma unroll
          for (int a = 1; a <= DS; a++) {
            const int k = rem % 3;
            rem /= 3;
            c += k == 0 ? off[a][0] : (k == 1 ? off[a][1] : off[a][2]);
          }
          xv[it] = *reinterpret_cast<const Ch *>(x + c * NC + jc * J);
        }
      }
#pragma unroll
      for (int it = 0; it < UNR; it++) {
        const int b = b0 + it * BPI;
        if (b < nb) acc = chunk_mac<T>(acc, v[it], xv[it]);
      }
    }
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    if (off & IMASK) continue;
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
  }
  if (row < nrows && lane == i * IB) {
    const int64_t o = row * NC + i;
    if (RESID) {
      cx<T> bb = bvec[o];
      y[o] = mk<cx<T>>(bb.x - acc.x, bb.y - acc.y);
    } else {
      y[o] = mk<cx<T>>(alpha * acc.x, alpha * acc.y);
    }
  }
}

// Row tiles of the LDS-staged kernel: RPW consecutive rows of one line of
// axis 1 (fixed tau and, for d = 2, fixed i_2).  Tiles per operator:
inline int64_t st_tiles(const Stencil &g, int rpw) {
  return (int64_t)g.nt * (g.S / g.n[1]) * ((g.n[1] + rpw - 1) / rpw);
}

// The structured SpMV with the x operand staged in LDS (2x2 blocks, d <= 2):
// the workgroup's rows share their time node and transverse coordinate, so
// all their neighbours lie in (time slices) x (3 transverse lines, d = 2) x
// (RPW + 2 consecutive nodes of axis 1); that tile is loaded once,
// cooperatively, while the value loads are in flight, and every block then
// reads its x chunk from LDS instead of gathering it from L2.  G lanes serve
// RPL consecutive rows (their value loads all issued before the first
// multiply), so a workgroup owns RPW = 256 / G * RPL rows.  Measured at 2+1D
// 128^3: 10 % faster than gathering x from L2; G = 16, RPL = 2 (complex128)
// and G = 8, RPL = 2 (complex64) a further 5-7 % over one row per 32 / 16
// lanes (76 % and 70 % of HBM peak).
template <typename T, int DS, int G, int RPL, bool RESID>
__device__ __forceinline__ void spmv_tile_lds(int64_t tile, const Stencil &g, const cx<T> *__restrict__ val,
                                              const cx<T> *__restrict__ x, const cx<T> *__restrict__ bvec,
                                              cx<T> *__restrict__ y, T alpha) {
  constexpr int NC = 2;
  using Ch = typename chunk_of<T>::type;
  constexpr int J = chunk_of<T>::J;
  constexpr int IB = NC / J;          // chunks per x node and per block row
  constexpr int CPB = NC * NC / J;    // chunks per block
  constexpr int BPI = G / CPB;        // blocks per group slice
  constexpr int RPW = 256 / G * RPL;  // rows per workgroup
  constexpr int IMASK = (NC - 1) * IB;
  constexpr int P = DS == 1 ? 3 : 9;
  constexpr int NY = DS == 1 ? 1 : 3;  // transverse lines
  constexpr int TW = RPW + 2;          // nodes of axis 1 per line
  constexpr int MAXB = 3 * P;
  constexpr int UNR = (MAXB + BPI - 1) / BPI;
  static_assert(G % CPB == 0 && G <= 64, "group must hold whole blocks");
  __shared__ Ch xs[3 * NY * TW * IB];
  const int n1 = g.n[1], n2 = DS == 2 ? g.n[2] : 1;
  const int tpl = (n1 + RPW - 1) / RPW;
  const int64_t line = tile / tpl;
  const int x0 = (int)(tile - line * tpl) * RPW;
  const int tau = (int)(line / n2) + 1;
  const int yy = (int)(line - (int64_t)(tau - 1) * n2);
  const int tau0 = tau >= 2 ? tau - 1 : tau;
  const int ntime = g.nt == 1 ? 1 : ((tau == 1 || tau == g.nt) ? 2 : 3);
  const int lane = threadIdx.x % G;
  const int xr0 = x0 + (int)(threadIdx.x / G) * RPL;  // first row of this lane group
  const int i = (lane / IB) % NC, jc = lane % IB, bofs = lane / CPB;
  // value loads first: their HBM latency overlaps the x staging
  Ch v[RPL][UNR];
  int nb[RPL];
#pragma unroll
  for (int r = 0; r < RPL; r++) {
    nb[r] = 0;
    if (xr0 + r < n1) {
      int64_t rs;
      st_row<DS>(g, line * n1 + xr0 + r, rs, nb[r]);
      const Ch *vbase = reinterpret_cast<const Ch *>(val + rs * NC * NC + i * NC + jc * J);
#pragma unroll
      for (int it = 0; it < UNR; it++) {
        const int b = bofs + it * BPI;
        if (b < nb[r]) {
          if constexpr (sizeof(T) == 8) v[r][it] = __builtin_nontemporal_load(vbase + (int64_t)b * CPB);
          else v[r][it] = vbase[(int64_t)b * CPB];
        }
      }
    }
  }
  // residual form: the right-hand side entries this lane writes are loaded
  // with the values, not after the products (a load issued at the end would
  // add one memory latency to every workgroup)
  cx<T> bpre[RPL];
#pragma unroll
  for (int r = 0; r < RPL; r++) {
    bpre[r] = mk<cx<T>>(0, 0);
    if (RESID && xr0 + r < n1 && lane == i * IB) bpre[r] = bvec[(line * n1 + xr0 + r) * NC + i];
  }
  // stage x: chunk e = ((kt NY + ly) TW + lx) IB + c
  for (int e = threadIdx.x; e < ntime * NY * TW * IB; e += 256) {
    const int c = e % IB, node = e / IB;
    const int lx = node % TW, ly = (node / TW) % NY, kt = node / (TW * NY);
    int xg = (x0 - 1 + lx) % n1;  // the tile can be wider than a short axis
    xg += xg < 0 ? n1 : 0;
    int yg = DS == 2 ? yy - 1 + ly : 0;
    if (DS == 2) {
      yg += yg < 0 ? n2 : 0;
      yg -= yg >= n2 ? n2 : 0;
    }
    const int64_t col = (int64_t)(tau0 + kt - 1) * g.S + (int64_t)yg * n1 + xg;
    xs[e] = *reinterpret_cast<const Ch *>(x + col * NC + c * J);
  }
  __syncthreads();
  // LDS slot of each sorted neighbour along axis 2 (shared by the workgroup)
  int lyk[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    int dy = 0;
    if (DS == 2) {
      dy = nb_coord(yy, n2, k) - (yy - 1);
      dy += dy < 0 ? n2 : 0;
      dy -= dy >= n2 ? n2 : 0;
    }
    lyk[k] = dy;
  }
#pragma unroll
  for (int r = 0; r < RPL; r++) {
    const int xr = xr0 + r;
    const bool own = xr < n1;
    cx<T> acc = mk<cx<T>>(0, 0);
    if (own) {
      // LDS slot of each sorted neighbour along axis 1 (inside the tile)
      int lxk[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        int d = nb_coord(xr, n1, k) - (x0 - 1);
        d += d < 0 ? n1 : 0;
        d -= d >= n1 ? n1 : 0;
        lxk[k] = d;
      }
#pragma unroll
      for (int it = 0; it < UNR; it++) {
        const int b = bofs + it * BPI;
        if (b < nb[r]) {
          const int kt = b / P, rem = b - kt * P;
          const int ky = DS == 2 ? rem / 3 : 0, kx = rem - ky * 3;
          const int lx = kx == 0 ? lxk[0] : (kx == 1 ? lxk[1] : lxk[2]);
          const int ly = ky == 0 ? lyk[0] : (ky == 1 ? lyk[1] : lyk[2]);
          acc = chunk_mac<T>(acc, v[r][it], xs[((kt * NY + ly) * TW + lx) * IB + jc]);
        }
      }
    }
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      if (off & IMASK) continue;
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (own && lane == i * IB) {
      const int64_t o = (line * n1 + xr) * NC + i;
      if (RESID) {
        y[o] = mk<cx<T>>(bpre[r].x - acc.x, bpre[r].y - acc.y);
      } else {
        y[o] = mk<cx<T>>(alpha * acc.x, alpha * acc.y);
      }
    }
  }
}

template <typename T, int DS, int G, int RPL, bool RESID>
__global__ __launch_bounds__(256) void spmv_lds_kernel(int64_t ntiles, Stencil g, const cx<T> *__restrict__ val,
                                                       const cx<T> *__restrict__ x,
                                                       const cx<T> *__restrict__ bvec,
                                                       cx<T> *__restrict__ y, T alpha) {
  spmv_tile_lds<T, DS, G, RPL, RESID>(xcd_tile(blockIdx.x, ntiles), g, val, x, bvec, y, alpha);
}

template <typename T, int NC, int DS, int G, bool RESID>
__global__ __launch_bounds__(256) void spmv_st_kernel(int64_t nrows, int64_t nwg, Stencil g,
                                                      const cx<T> *__restrict__ val,
                                                      const cx<T> *__restrict__ x,
                                                      const cx<T> *__restrict__ bvec,
                                                      cx<T> *__restrict__ y, T alpha) {
  spmv_tile_st<T, NC, DS, G, RESID>(xcd_tile(blockIdx.x, nwg), nrows, g, val, x, bvec, y, alpha);
}

template <typename T, int NC, int G, bool RESID>
__global__ __launch_bounds__(256) void spmv_kernel(int64_t nrows, int64_t nwg,
                                                   const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const cx<T> *__restrict__ val,
                                                   const cx<T> *__restrict__ x,
                                                   const cx<T> *__restrict__ bvec,
                                                   cx<T> *__restrict__ y, T alpha) {
  spmv_tile<T, NC, G, RESID>(xcd_tile(blockIdx.x, nwg), nrows, rp, ci, val, x, bvec, y, alpha);
}

// Host launcher: picks the group size for (T, nc).  resid: y = bvec - A x.
template <typename T>
inline hipError_t launch_spmv(int nc, int64_t nrows, const int32_t *rp, const int32_t *ci,
                              const void *val, const void *x, const void *bvec, void *y, T alpha,
                              bool resid, hipStream_t st) {
  auto go = [&](auto kern, int G) {
    const int64_t rpw = 256 / G;
    const int64_t nwg = (nrows + rpw - 1) / rpw;
    const int tk = kt_start(resid ? DIRAC_ST_TIMED_RESID64
                                  : (sizeof(T) == 8 ? DIRAC_ST_TIMED_SPMV64 : DIRAC_ST_TIMED_SPMV32), st);
    kern<<<(unsigned)nwg, 256, 0, st>>>(nrows, nwg, rp, ci, (const cx<T> *)val, (const cx<T> *)x,
                                        (const cx<T> *)bvec, (cx<T> *)y, alpha);
    kt_stop(tk, st);
    return hipGetLastError();
  };
  constexpr bool dbl = sizeof(T) == 8;
  if (nc == 2) {
    // lanes per 2x2 block row: the fastest of 4..64 measured on the 2+1D 128^3 operator
    constexpr int G = dbl ? 32 : 16;
    return resid ? go(spmv_kernel<T, 2, G, true>, G) : go(spmv_kernel<T, 2, G, false>, G);
  }
  constexpr int G4 = dbl ? 64 : 32;
  return resid ? go(spmv_kernel<T, 4, G4, true>, G4) : go(spmv_kernel<T, 4, G4, false>, G4);
}

// Host launcher for an operator built by dirac_st_assemble.  2x2 blocks use
// the structured kernel (no index traffic; measured 2 % faster in complex128
// and 20 % faster in complex64 than the indexed kernel at 2+1D 128^3); 4x4
// blocks keep the indexed kernel (its 16 lanes per block would all repeat the
// column arithmetic; 9 % slower structured at 3+1D 32^4).
template <typename T>
inline hipError_t launch_spmv_st(const dirac_st_bsr *A, const void *val, const void *x, const void *bvec,
                                 void *y, T alpha, bool resid, hipStream_t st) {
  if (A->nc == 4)
    return launch_spmv<T>(A->nc, A->nrows, A->row_ptr, A->col_idx, val, x, bvec, y, alpha, resid, st);
  const Stencil g = make_stencil(&A->prob);
  constexpr int RPL = 2;
  auto go = [&](auto kern, int G) {
    const int64_t ntiles = st_tiles(g, 256 / G * RPL);
    const int tk = kt_start(resid ? DIRAC_ST_TIMED_RESID64
                                  : (sizeof(T) == 8 ? DIRAC_ST_TIMED_SPMV64 : DIRAC_ST_TIMED_SPMV32), st);
    kern<<<(unsigned)ntiles, 256, 0, st>>>(ntiles, g, (const cx<T> *)val, (const cx<T> *)x,
                                           (const cx<T> *)bvec, (cx<T> *)y, alpha);
    kt_stop(tk, st);
    return hipGetLastError();
  };
  constexpr int G2 = sizeof(T) == 8 ? 16 : 8;
  if (g.d == 1)
    return resid ? go(spmv_lds_kernel<T, 1, G2, RPL, true>, G2) : go(spmv_lds_kernel<T, 1, G2, RPL, false>, G2);
  return resid ? go(spmv_lds_kernel<T, 2, G2, RPL, true>, G2) : go(spmv_lds_kernel<T, 2, G2, RPL, false>, G2);
}

}  // namespace dst
