// assemble.hip -- assembly of the spacetime Q1 Dirac operator into block CSR.
//
// The global block coupling row node r to column node c is the sum, over the
// elements that contain both nodes, of the element block
//     B_e(beta, alpha) = sum_mu i g^mu D^mu - m D^0 I - g^0 P
// (App. A, eq. (diracWeak1p1) extended per axis; Sec. 2.2 element summation).
// On a tensor mesh every element matrix is a product of 1D factors, one per
// axis, and the elements containing both nodes are the product of the 1D
// element choices per axis; so the sum over elements factorises into a product
// over axes of 1D sums.  Each GPU thread builds one block that way (a gather:
// no atomics, deterministic), writes it in complex128 and complex64, its
// column index, the row pointer and, for diagonal blocks, the inverse used by
// the node-block Jacobi preconditioner.
//
// Rows at t = 0 are not assembled; their columns form D_w21 and are applied
// to psi0 directly to give b = -D_w21 psi0 (Sec. 2.1, eq. (dirac_weakIVP)).
#include <cmath>

#include "common.hpp"

namespace dst {

struct AsmParams {
  int d, nc, nt;
  int n[4];
  int64_t S, nrows, nnzb;
  int64_t stride[4];   // spatial node strides (axis 1 fastest)
  double h[4];
  double M[4][2][2];   // 1D element mass  int phi_b phi_a     (row b = test)
  double Cd[4][2][2];  // 1D element       int phi_b phi_a'
  double m;
  int vkind;
  double v0, x0, lw;
  double2 g[4][16];    // gamma^mu, row-major nc x nc
  int c1, cint, clast, sp3;
  int64_t off_int, off_last;
};

static AsmParams make_params(const dirac_st_problem *p) {
  AsmParams P{};
  P.d = p->d;
  P.nc = p->nc;
  P.nt = p->n[0];
  for (int a = 0; a < 4; a++) P.n[a] = (a <= p->d) ? p->n[a] : 1;
  P.S = spatial_nodes(p);
  P.nrows = P.S * P.nt;
  P.nnzb = total_blocks(p);
  int64_t st = 1;
  P.stride[0] = 0;
  for (int a = 1; a < 4; a++) {
    P.stride[a] = st;
    if (a <= p->d) st *= p->n[a];
  }
  for (int a = 0; a < 4; a++) {
    double h = (a <= p->d) ? p->len[a] / p->n[a] : 1.0;
    P.h[a] = h;
    // closed forms of the 1D Q1 element integrals on [0, h]
    P.M[a][0][0] = P.M[a][1][1] = h / 3.0;
    P.M[a][0][1] = P.M[a][1][0] = h / 6.0;
    P.Cd[a][0][0] = P.Cd[a][1][0] = -0.5;
    P.Cd[a][0][1] = P.Cd[a][1][1] = 0.5;
  }
  P.m = p->m;
  P.vkind = p->vkind;
  P.v0 = p->v0;
  P.x0 = p->x0;
  P.lw = p->lw;
  gamma_set(p->d, P.g);
  P.sp3 = 1;
  for (int a = 0; a < p->d; a++) P.sp3 *= 3;
  P.c1 = blocks_per_row(p, 1);
  P.cint = blocks_per_row(p, 2 <= P.nt - 1 ? 2 : 1);
  P.clast = blocks_per_row(p, P.nt);
  P.off_int = P.S * P.c1;
  P.off_last = (P.nt >= 2) ? P.off_int + (int64_t)(P.nt - 2) * P.S * P.cint : P.off_int;
  return P;
}

// Streaming (nontemporal) stores for the bulk of what the assembly writes
// (values, column indices, right-hand side): none of it is read again before
// the solve, and plain stores would leave up to the whole memory-side cache
// dirty, to be written back during (and charged to) the solver's first
// bandwidth-bound kernels (measured: an SpMV right after a plain-store
// assembly takes 0.72 ms instead of 0.65 ms at 2+1D 128^3).  The node-block
// inverses (one 64-byte block per row, written by every 27th lane) stay plain:
// scattered partial-line streaming stores were slower.
__device__ inline void st_nt(double2 *p, double2 v) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  d2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<d2v *>(p));
}
__device__ inline void st_nt(float2 *p, float2 v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  f2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<f2v *>(p));
}
__device__ inline void st_nt(int32_t *p, int32_t v) { __builtin_nontemporal_store(v, p); }

__device__ inline double potential(const AsmParams &P, double x) {
  if (P.vkind == DIRAC_ST_V_STEP) return x > P.x0 ? P.v0 : 0.0;
  if (P.vkind == DIRAC_ST_V_SMOOTH) return 0.5 * P.v0 * (1.0 + tanh((x - P.x0) / P.lw));
  return 0.0;
}

// 2-point Gauss-Legendre: int_e V phi_b phi_a along axis 1, element e
__device__ inline double potential_weight(const AsmParams &P, int e, int b, int a) {
  const double h = P.h[1];
  const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
  double acc = 0.0;
  for (int q = 0; q < 2; q++) {
    double xi = 0.5 * (1.0 + (q ? r3 : -r3));
    double pb = b ? xi : 1.0 - xi, pa = a ? xi : 1.0 - xi;
    acc += 0.5 * h * potential(P, (e + xi) * h) * pb * pa;
  }
  return acc;
}

// Block coupling the row node with coordinates gr (gr[0] = time node tau) to
// the column node at offsets o (each -1, 0, +1).  DS = spatial dimensions
// (compile time, so every per-axis array stays in registers).
template <int NC, int DS>
__device__ void block_value(const AsmParams &P, const int *gr, const int *o, double2 *blk) {
  double KM[DS + 1], KC[DS + 1], KW = 0.0;
#pragma unroll
  for (int a = 0; a <= DS; a++) {
    const int n = P.n[a];
    double km = 0.0, kc = 0.0, kw = 0.0;
    // elements along axis a containing both nodes: offset +1 -> the row
    // node's element (local 0 -> 1); -1 -> the previous one (1 -> 0);
    // 0 -> both neighbouring elements (1 -> 1 and 0 -> 0)
#pragma unroll
    for (int c = 0; c < 2; c++) {
      int e, bb, aa;
      if (o[a] == 1) {
        if (c) continue;
        e = gr[a], bb = 0, aa = 1;
      } else if (o[a] == -1) {
        if (c) continue;
        e = gr[a] - 1, bb = 1, aa = 0;
      } else {
        e = c ? gr[a] : gr[a] - 1;
        bb = c ? 0 : 1;
        aa = bb;
      }
      if (a == 0) {
        if (e < 0 || e >= n) continue;
      } else {
        e = (e + n) % n;
      }
      km += P.M[a][bb][aa];
      kc += P.Cd[a][bb][aa];
      if (a == 1 && P.vkind != DIRAC_ST_V_NONE) kw += potential_weight(P, e, bb, aa);
    }
    KM[a] = km;
    KC[a] = kc;
    if (a == 1) KW = kw;
  }
  double Dmu[DS + 1], D0 = 1.0, Pw = KW;
#pragma unroll
  for (int mu = 0; mu <= DS; mu++) {
    double v = 1.0;
#pragma unroll
    for (int a = 0; a <= DS; a++) v *= (a == mu) ? KC[a] : KM[a];
    Dmu[mu] = v;
  }
#pragma unroll
  for (int a = 0; a <= DS; a++) {
    D0 *= KM[a];
    if (a != 1) Pw *= KM[a];
  }
#pragma unroll
  for (int i = 0; i < NC; i++)
#pragma unroll
    for (int j = 0; j < NC; j++) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int mu = 0; mu <= DS; mu++) {
        double2 gg = P.g[mu][i * NC + j];
        re -= gg.y * Dmu[mu];  // i * g
        im += gg.x * Dmu[mu];
      }
      if (i == j) re -= P.m * D0;
      double2 g0 = P.g[0][i * NC + j];
      re -= g0.x * Pw;
      im -= g0.y * Pw;
      blk[i * NC + j] = mk<double2>(re, im);
    }
}

// sorted neighbour offset of digit k along a periodic axis of length n (n >= 3)
__device__ inline int spatial_offset(int i, int n, int k) {
  if (i == 0) return k == 0 ? 0 : (k == 1 ? 1 : -1);
  if (i == n - 1) return k == 0 ? 1 : (k == 1 ? -1 : 0);
  return k - 1;
}

// Gauss-Jordan inverse with partial pivoting; returns false if singular or if
// the 1-norm condition number exceeds 1e12.  Row swaps are unrolled selects.
template <int NC>
__device__ bool block_inverse(const double2 *a, double2 *inv) {
  double2 m[NC][2 * NC];
  double na = 0.0;
#pragma unroll
  for (int j = 0; j < NC; j++) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NC; i++) s += sqrt(cabs2(a[i * NC + j]));
    na = fmax(na, s);
  }
#pragma unroll
  for (int i = 0; i < NC; i++)
#pragma unroll
    for (int j = 0; j < 2 * NC; j++)
      m[i][j] = (j < NC) ? a[i * NC + j] : mk<double2>(j - NC == i ? 1.0 : 0.0, 0.0);
  bool ok = true;
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
    if (best == 0.0) ok = false;
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
    double dd = best > 0.0 ? 1.0 / cabs2(d) : 0.0;
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
  double ni = 0.0;
#pragma unroll
  for (int j = 0; j < NC; j++) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NC; i++) s += sqrt(cabs2(m[i][NC + j]));
    ni = fmax(ni, s);
  }
#pragma unroll
  for (int i = 0; i < NC; i++)
#pragma unroll
    for (int j = 0; j < NC; j++) inv[i * NC + j] = m[i][NC + j];
  return ok && na * ni <= 1e12 && isfinite(na * ni);
}

// Block kb of the CSR value array: its row, position k in the row, column
// node, whether it is the diagonal block, and its values.
template <int NC, int DS>
__device__ inline void block_at(const AsmParams &P, int64_t kb, int64_t &r, int &k,
                                int64_t &colnode, bool &diag, double2 *blk) {
  int tau, c;
  int64_t s;
  if (kb < P.off_int) {
    tau = 1;
    c = P.c1;
    s = kb / c;
    k = (int)(kb - s * c);
  } else if (kb < P.off_last) {
    int64_t q = kb - P.off_int, per = P.S * P.cint;
    int64_t sl = q / per;
    tau = 2 + (int)sl;
    q -= sl * per;
    c = P.cint;
    s = q / c;
    k = (int)(q - s * c);
  } else {
    int64_t q = kb - P.off_last;
    tau = P.nt;
    c = P.clast;
    s = q / c;
    k = (int)(q - s * c);
  }
  r = (int64_t)(tau - 1) * P.S + s;
  int gr[DS + 1], o[DS + 1];
  gr[0] = tau;
  int64_t ss = s;
#pragma unroll
  for (int a = 1; a <= DS; a++) {
    gr[a] = (int)(ss % P.n[a]);
    ss /= P.n[a];
  }
  // block position k -> offsets: time slowest, then axis d ... axis 1; the
  // time neighbours present are tau-1 (if tau >= 2), tau, tau+1 (if tau < n_t)
  const int kt = k / P.sp3;
  int ks = k - kt * P.sp3;
  o[0] = kt - (tau >= 2 ? 1 : 0);
  colnode = (int64_t)(tau + o[0] - 1) * P.S;
  diag = (o[0] == 0);
#pragma unroll
  for (int a = 1; a <= DS; a++) {
    const int dig = ks % 3;
    ks /= 3;
    o[a] = spatial_offset(gr[a], P.n[a], dig);
    colnode += (int64_t)((gr[a] + o[a] + P.n[a]) % P.n[a]) * P.stride[a];
    diag = diag && (o[a] == 0);
  }
  block_value<NC, DS>(P, gr, o, blk);
}

// One thread per stored block.  The workgroup's blocks form one contiguous
// stretch of the value arrays, so they are staged in LDS and written out with
// consecutive lanes on consecutive 16-byte (complex128) entries.
template <int NC, int DS, int BS>
__global__ __launch_bounds__(BS) void assemble_kernel(AsmParams P, int32_t *__restrict__ row_ptr,
                                                       int32_t *__restrict__ col_idx,
                                                       double2 *__restrict__ val64,
                                                       float2 *__restrict__ val32,
                                                       double2 *__restrict__ bj64,
                                                       float2 *__restrict__ bj32,
                                                       int32_t *__restrict__ nsingular) {
  // staging of the blocks for coalesced stores.  4x4 blocks: entry-major with
  // one pad slot per entry row, so that the per-thread writes (fixed entry,
  // consecutive blocks) do not all hit one bank (measured 6 % faster at 3+1D
  // 32^4); 2x2 blocks: block-major (faster at 2+1D 128^3)
  constexpr int LS = BS + 1;
  __shared__ double2 sblk[NC == 4 ? NC * NC * LS : NC * NC * BS];
  __shared__ int32_t scol[BS];
  auto slot = [&](int t, int q) { return NC == 4 ? q * LS + t : t * NC * NC + q; };
  const int64_t kb0 = (int64_t)blockIdx.x * BS;
  const int64_t kb = kb0 + threadIdx.x;
  if (kb < P.nnzb) {
    int64_t r, colnode;
    int k;
    bool diag;
    double2 blk[NC * NC];
    block_at<NC, DS>(P, kb, r, k, colnode, diag, blk);
#pragma unroll
    for (int q = 0; q < NC * NC; q++) sblk[slot(threadIdx.x, q)] = blk[q];
    scol[threadIdx.x] = (int32_t)colnode;
    if (k == 0) row_ptr[r] = (int32_t)kb;
    if (kb == P.nnzb - 1) row_ptr[P.nrows] = (int32_t)P.nnzb;
    if (diag && bj64) {
      double2 inv[NC * NC];
      if (!block_inverse<NC>(blk, inv)) {
        atomicAdd(nsingular, 1);
#pragma unroll
        for (int i = 0; i < NC; i++)
#pragma unroll
          for (int j = 0; j < NC; j++) inv[i * NC + j] = mk<double2>(i == j ? 1.0 : 0.0, 0.0);
      }
      double2 *b64 = bj64 + r * NC * NC;
#pragma unroll
      for (int q = 0; q < NC * NC; q++) b64[q] = inv[q];
      if (bj32) {
        float2 *b32 = bj32 + r * NC * NC;
#pragma unroll
        for (int q = 0; q < NC * NC; q++) b32[q] = to32(inv[q]);
      }
    }
  }
  __syncthreads();
  const int64_t nb = (P.nnzb - kb0) < BS ? (P.nnzb - kb0) : BS;
  const int nent = (int)nb * NC * NC;
  double2 *v64 = val64 + kb0 * NC * NC;
  for (int e = threadIdx.x; e < nent; e += BS) st_nt(v64 + e, sblk[slot(e / (NC * NC), e % (NC * NC))]);
  // column indices four to a lane (whole 16-byte pieces; kb0 is a multiple of BS)
  if (nb == BS) {
    typedef int i4v __attribute__((ext_vector_type(4)));
    if (threadIdx.x < BS / 4) {
      i4v c;
      c.x = scol[4 * threadIdx.x];
      c.y = scol[4 * threadIdx.x + 1];
      c.z = scol[4 * threadIdx.x + 2];
      c.w = scol[4 * threadIdx.x + 3];
      __builtin_nontemporal_store(c, reinterpret_cast<i4v *>(col_idx + kb0) + threadIdx.x);
    }
  } else if (threadIdx.x < nb) {
    st_nt(col_idx + kb0 + threadIdx.x, scol[threadIdx.x]);
  }
  if (val32) {
    float2 *v32 = val32 + kb0 * NC * NC;
    for (int e = threadIdx.x; e < nent; e += BS) st_nt(v32 + e, to32(sblk[slot(e / (NC * NC), e % (NC * NC))]));
  }
}

__global__ void zero_i32(int32_t *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// b = -D_w21 psi0: only rows of the first time slice see the t = 0 columns.
template <int NC, int DS>
__global__ __launch_bounds__(256) void rhs_kernel(AsmParams P, const double2 *__restrict__ psi0,
                                                   double2 *__restrict__ b) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= P.nrows) return;
  double2 acc[NC];
#pragma unroll
  for (int i = 0; i < NC; i++) acc[i] = mk<double2>(0, 0);
  if (r < P.S) {
    int gr[DS + 1], o[DS + 1];
    gr[0] = 1;
    o[0] = -1;
    int64_t ss = r;
#pragma unroll
    for (int a = 1; a <= DS; a++) {
      gr[a] = (int)(ss % P.n[a]);
      ss /= P.n[a];
    }
    for (int ks = 0; ks < P.sp3; ks++) {
      int t = ks;
      int64_t col = 0;
#pragma unroll
      for (int a = 1; a <= DS; a++) {
        o[a] = (t % 3) - 1;
        t /= 3;
        col += (int64_t)((gr[a] + o[a] + P.n[a]) % P.n[a]) * P.stride[a];
      }
      double2 blk[NC * NC];
      block_value<NC, DS>(P, gr, o, blk);
#pragma unroll
      for (int i = 0; i < NC; i++)
#pragma unroll
        for (int j = 0; j < NC; j++) acc[i] = cfma(acc[i], blk[i * NC + j], psi0[col * NC + j]);
    }
  }
#pragma unroll
  for (int i = 0; i < NC; i++) st_nt(b + r * NC + i, mk<double2>(-acc[i].x, -acc[i].y));
}

}  // namespace dst

using namespace dst;

extern "C" int dirac_st_assemble(const dirac_st_problem *prob, const void *psi0, dirac_st_bsr *A,
                                 void *b, void *stream) {
  clear_error();
  if (int rc = validate_problem(prob)) return rc;
  DST_CHECK(A && A->row_ptr && A->col_idx && A->val64, "matrix arrays must be set");
  DST_CHECK(!b || psi0, "psi0 is required to form b");
  AsmParams P = make_params(prob);
  DST_CHECK(A->nrows == P.nrows && A->nnzb == P.nnzb,
            "A->nrows/nnzb (%lld/%lld) differ from dirac_st_sizes (%lld/%lld)",
            (long long)A->nrows, (long long)A->nnzb, (long long)P.nrows, (long long)P.nnzb);
  hipStream_t st = (hipStream_t)stream;
  int32_t *dsing = nullptr;
  if (A->bjinv64) {
    DST_HIP(hipMallocAsync((void **)&dsing, sizeof(int32_t), st));
    zero_i32<<<1, 64, 0, st>>>(dsing, 1);
    DST_LAUNCHED();
  }
  const unsigned g256 = (unsigned)((P.nnzb + 255) / 256);
  const unsigned grow = (unsigned)((P.nrows + 255) / 256);
  double2 *v64 = (double2 *)A->val64, *bj64 = (double2 *)A->bjinv64;
  float2 *v32 = (float2 *)A->val32, *bj32 = (float2 *)A->bjinv32;
  const double2 *ps = (const double2 *)psi0;
  double2 *bb = (double2 *)b;
  const int tk = kt_start(DIRAC_ST_TIMED_ASSEMBLE, st);
  if (P.d == 1) {
    assemble_kernel<2, 1, 256><<<g256, 256, 0, st>>>(P, A->row_ptr, A->col_idx, v64, v32, bj64, bj32, dsing);
    kt_stop(tk, st);
    if (b) rhs_kernel<2, 1><<<grow, 256, 0, st>>>(P, ps, bb);
  } else if (P.d == 2) {
    assemble_kernel<2, 2, 256><<<g256, 256, 0, st>>>(P, A->row_ptr, A->col_idx, v64, v32, bj64, bj32, dsing);
    kt_stop(tk, st);
    if (b) rhs_kernel<2, 2><<<grow, 256, 0, st>>>(P, ps, bb);
  } else {
    assemble_kernel<4, 3, 128><<<(unsigned)((P.nnzb + 127) / 128), 128, 0, st>>>(
        P, A->row_ptr, A->col_idx, v64, v32, bj64, bj32, dsing);
    kt_stop(tk, st);
    if (b) rhs_kernel<4, 3><<<grow, 256, 0, st>>>(P, ps, bb);
  }
  DST_LAUNCHED();
  A->nc = prob->nc;
  A->prob = *prob;
  A->singular_blocks = 0;
  if (dsing) {
    int32_t h = 0;
    DST_HIP(hipMemcpyAsync(&h, dsing, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DST_HIP(hipFreeAsync(dsing, st));
    DST_HIP(hipStreamSynchronize(st));
    A->singular_blocks = h;
  }
  return DIRAC_ST_OK;
}
