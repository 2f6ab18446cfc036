// batched.hip -- flexible GMRES(m) over many independent systems of uneven
// size in grouped launches.
//
// Every active system advances through the same Arnoldi step j together.  Each
// phase of the step -- preconditioner, SpMV, the three Gram-Schmidt passes,
// the reductions, the Givens update -- is ONE launch for the whole batch: the
// grid walks a device work list of (system, tile) items and each workgroup
// reads its system's descriptor (operator, basis, partial sums, FP64 cycle
// state) before running the same per-tile code as the single-system solver.
// A system whose residual estimate meets the tolerance (or whose cycle ends on
// a happy breakdown) drops out of the lists for the rest of the cycle; after
// each cycle its FP64 true residual decides whether it retires.  Like the
// single-system solver, inner cycles may run in complex64 (SpMV on val32, basis
// in complex64) under FP64 refinement: every cycle starts from b - A x in
// complex128 and adds its correction x += Z y in FP64.
//
// The SpMV tile (lanes per block row) is chosen by an autotuner: the first
// call for a (block size, precision, batch size class) times each candidate
// on the batch itself with HIP events and caches the fastest.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "krylov.hpp"
#include "precond.hpp"
#include "readback.hpp"
#include "spectral.hpp"
#include "spmv.hpp"

namespace dst {

// lane code of the x-staged line-tile SpMV (2x2 blocks) and its rows per
// workgroup (see g_spmv); codes 4..64 are lanes per block row of the gather
// kernels
constexpr int kLdsLanes = 1;
constexpr int kLdsRows = 32;

struct BSys {
  const int32_t *rp, *ci;
  const void *val64, *val32, *bj64, *bj32;
  int64_t nrows, n, nblk, ldv;
  void *V;       // m+1 basis vectors, working precision
  void *Z;       // m preconditioned vectors, working precision
  double2 *r64;  // FP64 residual
  double2 *x;
  const double2 *b;
  double2 *partial;  // [64][nblk]
  Ctrl *ctrl;
  int nc, k;     // block size; steps of the current cycle (set before updates)
  int64_t lt[4]; // line preconditioner workgroups: time transform, axis 2, axis 3, line solve
  Stencil st;    // block-row structure (2x2 blocks: the SpMV reads no indices)
};

// Line preconditioner of one system (device copy; pointers at the working precision).
struct LineJob {
  const void *Q, *W, *F[4], *Fi[4];
  void *b1, *b2;
  const void *fac, *lined;
  int pk, pm, dpk[4], dpm[4];
  int d, nc, nt, n[4];
  int64_t S, lines;
};

constexpr int kMaxBatch = DIRAC_ST_MAX_BATCH;

// Work lists of one launch: the grid's workgroups are numbered 0..off[nact]-1
// and system act[a] owns workgroups [off[a], off[a+1]).  tab[w] = a for every
// workgroup w (filled on the device whenever the list changes), so a
// workgroup finds its system with two scalar loads.  The XCD-aware
// renumbering keeps the tiles an XCD processes contiguous (one system's rows
// share that XCD's L2).
struct WorkList {
  const int64_t *act;   // active systems
  const int64_t *off;   // nact + 1 prefix sums of workgroups per system
  const uint16_t *tab;  // position in act of each workgroup's system
  int nact;
};

__device__ __forceinline__ int find_sys(const WorkList &L, int64_t &local) {
  const int64_t bid = xcd_tile(blockIdx.x, gridDim.x);
  // every lane holds the same values: make that visible to the compiler so
  // the descriptor fields and everything derived from them stay scalar
  const int a = __builtin_amdgcn_readfirstlane((int)L.tab[bid]);
  const int64_t loc = bid - L.off[a];
  const int lo32 = __builtin_amdgcn_readfirstlane((int)(uint32_t)(loc & 0xffffffff));
  const int hi32 = __builtin_amdgcn_readfirstlane((int)(loc >> 32));
  local = ((int64_t)hi32 << 32) | (uint32_t)lo32;
  return __builtin_amdgcn_readfirstlane((int)L.act[a]);
}

// tab[off[a] .. off[a+1]) = a, one workgroup per listed system
__global__ __launch_bounds__(256) void g_fill_tab(const int64_t *__restrict__ off, uint16_t *__restrict__ tab) {
  const int a = blockIdx.x;
  const int64_t e0 = off[a], e1 = off[a + 1];
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) tab[e] = (uint16_t)a;
}

// ------------------------------------------------------------ grouped kernels
// mode 0: V_{j+1} = A Z_j (working precision); mode 1: r64 = b - A x (FP64)
// G = kLdsLanes selects the x-staged line-tile kernel (2x2 blocks): 16 lanes
// per complex128 row serving 2 rows, 8 lanes per complex64 row serving 1 row,
// kLdsRows rows per workgroup in both precisions.
template <typename T, int NC, int G, int MODE>
__global__ __launch_bounds__(256) void g_spmv(const BSys *__restrict__ S, WorkList L, int j) {
  int64_t tile;
  const BSys &s = S[find_sys(L, tile)];
  if constexpr (NC == 2 && G == kLdsLanes) {
    constexpr int GL = sizeof(T) == 8 ? 16 : 8, RPL = kLdsRows * GL / 256;
    if (MODE == 0) {
      const cx<T> *z = (const cx<T> *)s.Z + (int64_t)j * s.ldv;
      cx<T> *w = (cx<T> *)s.V + (int64_t)(j + 1) * s.ldv;
      const cx<T> *val = (const cx<T> *)(sizeof(T) == 8 ? s.val64 : s.val32);
      if (s.st.d == 1) spmv_tile_lds<T, 1, GL, RPL, false>(tile, s.st, val, z, nullptr, w, (T)1);
      else spmv_tile_lds<T, 2, GL, RPL, false>(tile, s.st, val, z, nullptr, w, (T)1);
    } else {
      const double2 *val = (const double2 *)s.val64;
      if (s.st.d == 1) spmv_tile_lds<double, 1, 16, 2, true>(tile, s.st, val, s.x, s.b, s.r64, 1.0);
      else spmv_tile_lds<double, 2, 16, 2, true>(tile, s.st, val, s.x, s.b, s.r64, 1.0);
    }
  } else {
    if (MODE == 0) {
      const cx<T> *z = (const cx<T> *)s.Z + (int64_t)j * s.ldv;
      cx<T> *w = (cx<T> *)s.V + (int64_t)(j + 1) * s.ldv;
      const cx<T> *val = (const cx<T> *)(sizeof(T) == 8 ? s.val64 : s.val32);
      if constexpr (NC == 2) {
        if (s.st.d == 1) spmv_tile_st<T, 2, 1, G, false>(tile, s.nrows, s.st, val, z, nullptr, w, (T)1);
        else spmv_tile_st<T, 2, 2, G, false>(tile, s.nrows, s.st, val, z, nullptr, w, (T)1);
      } else {
        spmv_tile<T, NC, G, false>(tile, s.nrows, s.rp, s.ci, val, z, nullptr, w, (T)1);
      }
    } else {
      const double2 *val = (const double2 *)s.val64;
      if constexpr (NC == 2) {
        if (s.st.d == 1) spmv_tile_st<double, 2, 1, G, true>(tile, s.nrows, s.st, val, s.x, s.b, s.r64, 1.0);
        else spmv_tile_st<double, 2, 2, G, true>(tile, s.nrows, s.st, val, s.x, s.b, s.r64, 1.0);
      } else {
        spmv_tile<double, NC, G, true>(tile, s.nrows, s.rp, s.ci, val, s.x, s.b, s.r64, 1.0);
      }
    }
  }
}

template <typename T, int MAXK, int MODE>
__global__ __launch_bounds__(256) void g_cgs(const BSys *__restrict__ S, WorkList L, int jp1) {
  int64_t blk;
  const BSys &s = S[find_sys(L, blk)];
  cx<T> *V = (cx<T> *)s.V;
  cgs_block<T, MAXK, MODE>(blk, s.nblk, V, s.ldv, jp1, V + (int64_t)jp1 * s.ldv, s.ctrl->coef,
                           s.partial, s.n);
}

// partial[0][b] = |r64|^2 (src 0), |b|^2 (src 1) or |x|^2 (src 2) over the block
__global__ __launch_bounds__(256) void g_norm(const BSys *__restrict__ S, WorkList L, int src) {
  __shared__ double red[4];
  int64_t blk;
  const BSys &s = S[find_sys(L, blk)];
  const int64_t e = blk * 256 + threadIdx.x;
  double v = 0.0;
  if (e < s.n) v = cabs2(src == 0 ? s.r64[e] : src == 1 ? s.b[e] : s.x[e]);
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) s.partial[blk] = mk<double2>(red[0] + red[1] + red[2] + red[3], 0.0);
}

// blockIdx.y -> active system, blockIdx.x -> coefficient
__global__ __launch_bounds__(256) void g_reduce(const BSys *__restrict__ S, const int64_t *__restrict__ act,
                                                int what, int which) {
  const BSys &s = S[act[blockIdx.y]];
  reduce_coef(blockIdx.x, s.partial, s.nblk, s.ctrl, what, which);
}

// one workgroup per active system
__global__ void g_cycle_init(const BSys *__restrict__ S, const int64_t *__restrict__ act) {
  const BSys &s = S[act[blockIdx.x]];
  cycle_init_dev(s.ctrl, sqrt(s.ctrl->dots_norm2), 1.0);
}
__global__ void g_givens(const BSys *__restrict__ S, const int64_t *__restrict__ act, int j) {
  givens_dev(S[act[blockIdx.x]].ctrl, j);
}
__global__ void g_backsub(const BSys *__restrict__ S, const int64_t *__restrict__ act) {
  const BSys &s = S[act[blockIdx.x]];
  backsub_dev(s.ctrl, s.k, 1);
}

// V_0 = T(r64 / ||r64||)
template <typename T>
__global__ __launch_bounds__(256) void g_v0(const BSys *__restrict__ S, WorkList L) {
  int64_t blk;
  const BSys &s = S[find_sys(L, blk)];
  const int64_t e = blk * 256 + threadIdx.x;
  if (e >= s.n) return;
  const double inv = 1.0 / sqrt(s.ctrl->dots_norm2);
  const double2 v = s.r64[e];
  ((cx<T> *)s.V)[e] = mk<cx<T>>((T)(v.x * inv), (T)(v.y * inv));
}

// Z_j = sigma_j B^{-1} V_j (node-block Jacobi) or sigma_j V_j (no preconditioner)
template <typename T, int NC, bool BJ>
__global__ __launch_bounds__(256) void g_pc_local(const BSys *__restrict__ S, WorkList L, int j) {
  int64_t blk;
  const BSys &s = S[find_sys(L, blk)];
  const int64_t e = blk * 256 + threadIdx.x;
  if (e >= s.n) return;
  const T sg = (T)s.ctrl->sigma[j];
  const cx<T> *v = (const cx<T> *)s.V + (int64_t)j * s.ldv;
  cx<T> *z = (cx<T> *)s.Z + (int64_t)j * s.ldv;
  if (!BJ) {
    z[e] = mk<cx<T>>(v[e].x * sg, v[e].y * sg);
    return;
  }
  const cx<T> *binv = (const cx<T> *)(sizeof(T) == 8 ? s.bj64 : s.bj32);
  const int64_t r = e / NC;
  const int i = (int)(e - r * NC);
  cx<T> acc = mk<cx<T>>(0, 0);
#pragma unroll
  for (int q = 0; q < NC; q++) acc = cfma(acc, binv[(r * NC + i) * NC + q], v[r * NC + q]);
  z[e] = mk<cx<T>>(acc.x * sg, acc.y * sg);
}

// One transform of the line preconditioner for every listed system.
// axis 0: along time (Q, or W when dst == 3); axis a >= 2: transverse DFT
// (inverse if inv).  src/dst: 0 V_j, 1 b1, 2 b2, 3 Z_j.  The W transform
// scales by sigma_j (the stored V_j is sigma_j^{-1} times the basis vector).
// grid (x: tiles of the largest system, y: active systems).  AXIS 0: along
// time (Q, or sigma_j W when DST == 3); AXIS 2, 3: transverse DFT (inverse if
// INV).  SRC/DST: 0 V_j, 1 b1, 2 b2, 3 Z_j.
template <typename T, int AXIS, bool INV, int SRC, int DST>
__global__ __launch_bounds__(256) void g_line_gemm(const BSys *__restrict__ S, const LineJob *__restrict__ J,
                                                   const int64_t *__restrict__ act, int j) {
  const int sys = (int)act[blockIdx.y];
  const BSys &s = S[sys];
  if ((int64_t)blockIdx.x >= s.lt[AXIS == 0 ? 0 : AXIS - 1]) return;
  const LineJob &q = J[sys];
  using C = cx<T>;
  const C *A;
  int pk, pm, n;
  int64_t cols, batches = 1;
  if (AXIS == 0) {
    A = (const C *)(DST == 3 ? q.W : q.Q);
    pk = q.pk;
    pm = q.pm;
    n = q.nt;
    cols = q.S * q.nc;
  } else {
    A = (const C *)(INV ? q.Fi[AXIS] : q.F[AXIS]);
    pk = q.dpk[AXIS];
    pm = q.dpm[AXIS];
    n = q.n[AXIS];
    cols = q.nc;
    for (int b = 1; b < AXIS; b++) cols *= q.n[b];
  }
  (void)batches;
  // 32-bit index arithmetic: every count here is below 2^31 (grid limit)
  const unsigned nct = (unsigned)((cols + 63) / 64), nrt = (unsigned)(pm / 64), t32 = blockIdx.x;
  const unsigned ct = t32 % nct, rt = (t32 / nct) % nrt, bt = t32 / (nct * nrt);
  const C *X = SRC == 0 ? (const C *)s.V + (int64_t)j * s.ldv : (const C *)(SRC == 1 ? q.b1 : q.b2);
  C *Y = DST == 3 ? (C *)s.Z + (int64_t)j * s.ldv : (C *)(DST == 1 ? q.b1 : q.b2);
  const int64_t boff = (int64_t)bt * n * cols;
  const T scale = DST == 3 ? (T)s.ctrl->sigma[j] : (T)1;
  tgemm_tile<T>(A, pk, X + boff, Y + boff, n, cols, (int)rt * 64, (int64_t)ct * 64, scale);
}

// launches one transform of the line preconditioner (template dispatch)
template <typename T>
static void launch_line_gemm(int axis, bool inv, int src, int dst, dim3 grid, const BSys *S, const LineJob *J,
                             const int64_t *act, int j, hipStream_t st) {
  if (axis == 0) {
    if (dst == 3) {
      if (src == 1) g_line_gemm<T, 0, false, 1, 3><<<grid, 256, 0, st>>>(S, J, act, j);
      else g_line_gemm<T, 0, false, 2, 3><<<grid, 256, 0, st>>>(S, J, act, j);
    } else {
      g_line_gemm<T, 0, false, 0, 1><<<grid, 256, 0, st>>>(S, J, act, j);
    }
    return;
  }
#define DST_LG(AX)                                                                           \
  if (axis == AX) {                                                                          \
    if (inv) {                                                                               \
      if (src == 1) g_line_gemm<T, AX, true, 1, 2><<<grid, 256, 0, st>>>(S, J, act, j);       \
      else g_line_gemm<T, AX, true, 2, 1><<<grid, 256, 0, st>>>(S, J, act, j);               \
    } else {                                                                                 \
      if (src == 1) g_line_gemm<T, AX, false, 1, 2><<<grid, 256, 0, st>>>(S, J, act, j);      \
      else g_line_gemm<T, AX, false, 2, 1><<<grid, 256, 0, st>>>(S, J, act, j);              \
    }                                                                                        \
  }
  DST_LG(2)
  DST_LG(3)
#undef DST_LG
}

// Factorisation of the line preconditioner of every system in one launch.
struct LineSetupJob {
  SpecGeom G;
  const double2 *tw, *lam;
  const double *pot;
  void *fac, *lined;
  int64_t lines;
  int *flag;
};

// the line-setup flags of all systems into one array (one read-back)
__global__ void g_line_flags(const LineSetupJob *__restrict__ J, int nsys, int *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsys) out[i] = *J[i].flag;
}

template <typename T, int NC, int DS>
__global__ __launch_bounds__(64) void g_line_setup(const LineSetupJob *__restrict__ J, WorkList L) {
  int64_t tile;
  const LineSetupJob &q = J[find_sys(L, tile)];
  const int64_t l = tile * 64 + threadIdx.x;
  if (l < q.lines)
    line_setup_one<T, NC, DS>(q.G, q.tw, q.lam, q.pot, (cx<T> *)q.fac, (cx<T> *)q.lined, q.lines, q.flag, l);
}

template <typename T, int NC>
__global__ __launch_bounds__(64) void g_line_solve(const LineJob *__restrict__ J, WorkList L, int buf) {
  int64_t tile;
  const LineJob &q = J[find_sys(L, tile)];
  line_solve_wg<T, NC, kLineChunk>((const cx<T> *)q.fac, (const cx<T> *)q.lined,
                                   (cx<T> *)(buf == 1 ? q.b1 : q.b2), q.n[1], q.lines, tile * 64);
}

// x += sum_{i < k} Z_i coef_i (FP64 accumulation)
template <typename T>
__global__ __launch_bounds__(256) void g_update(const BSys *__restrict__ S, WorkList L) {
  int64_t blk;
  const BSys &s = S[find_sys(L, blk)];
  const int64_t e = blk * 256 + threadIdx.x;
  if (e >= s.n) return;
  double2 acc = s.x[e];
  const cx<T> *Z = (const cx<T> *)s.Z;
  const double2 *coef = s.ctrl->coef;
  for (int i = 0; i < s.k; i++) acc = cfma(acc, to64(Z[(int64_t)i * s.ldv + e]), coef[i]);
  s.x[e] = acc;
}

// r64 = b (the residual of the zero initial guess)
__global__ __launch_bounds__(256) void g_copy_b(const BSys *__restrict__ S, WorkList L) {
  int64_t blk;
  const BSys &s = S[find_sys(L, blk)];
  const int64_t e = blk * 256 + threadIdx.x;
  if (e < s.n) s.r64[e] = s.b[e];
}

// which = 0: Z_0 = 0 (working precision); which = 1: x = 0
template <typename T>
__global__ __launch_bounds__(256) void g_zero(const BSys *__restrict__ S, WorkList L, int which) {
  int64_t blk;
  const BSys &s = S[find_sys(L, blk)];
  const int64_t e = blk * 256 + threadIdx.x;
  if (e >= s.n) return;
  if (which == 0) ((cx<T> *)s.Z)[e] = mk<cx<T>>(0, 0);
  else s.x[e] = mk<double2>(0, 0);
}

// per-system read-back: est_abs, happy, finite, sigma_next, norm^2
__global__ void g_gather(const BSys *__restrict__ S, const int64_t *__restrict__ act, int nact,
                         double *__restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nact) return;
  const Ctrl *c = S[act[a]].ctrl;
  out[5 * a + 0] = c->est_abs;
  out[5 * a + 1] = c->happy;
  out[5 * a + 2] = c->finite;
  out[5 * a + 3] = c->sigma_next;
  out[5 * a + 4] = c->dots_norm2;
}

__global__ void g_zero_ctrl(const BSys *__restrict__ S) {
  double *p = reinterpret_cast<double *>(S[blockIdx.y].ctrl);
  const int64_t n = sizeof(Ctrl) / sizeof(double);
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

// ------------------------------------------------------------ host side
// work-list arrays: active systems, SpMV tiles, residual SpMV tiles, vector
// blocks, and the four line-preconditioner phases
constexpr int kListArrays = 8;

struct BatchLayout {
  std::vector<size_t> V, Z, r64, partial, ctrl, spec;
  std::vector<int64_t> ldv, nblk;
  size_t desc, jobs, sjobs, lists, gather, tab_w, tab_r, tab_v, tab_l, total;
  int64_t cap_rows, cap_vec, cap_lines;  // workgroup-table capacities
};

// fewest block rows one SpMV workgroup may cover (largest lane count)
static int64_t rows_per_wg_min(int nc) { return nc == 2 ? 256 / 32 : 256 / 64; }

// SpMV workgroups of one system for lane count g (kLdsLanes: line tiles)
static int64_t spmv_wgs(const BSys &q, int g) {
  if (g == kLdsLanes) return st_tiles(q.st, kLdsRows);
  const int64_t rw = 256 / g;
  return (q.nrows + rw - 1) / rw;
}

// table capacity for any lane count of this operator
static int64_t spmv_wgs_cap(const dirac_st_bsr *A) {
  int64_t c = (A->nrows + rows_per_wg_min(A->nc) - 1) / rows_per_wg_min(A->nc);
  if (A->nc == 2) c = std::max(c, st_tiles(make_stencil(&A->prob), kLdsRows));
  return c;
}

static BatchLayout batch_layout(int nsys, const dirac_st_bsr *const *A, const dirac_st_opts *o) {
  BatchLayout L;
  const size_t cs = o->precision == 32 ? 8 : 16;
  const int m = o->restart;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t r = off;
    off += align256(b);
    return r;
  };
  for (int i = 0; i < nsys; i++) {
    const int64_t N = A[i]->nrows * A[i]->nc;
    // consecutive vectors skewed by 4 KB: a power-of-two stride between the
    // streams that a pass reads together measured 5-10 % slower
    const size_t vb = align256((size_t)N * cs) + kVecSkew;
    L.ldv.push_back((int64_t)(vb / cs));
    L.nblk.push_back((N + 255) / 256);
    L.V.push_back(take(vb * (m + 1)));
    L.Z.push_back(take(vb * m));
    L.r64.push_back(take((size_t)N * 16));
    L.partial.push_back(take((size_t)L.nblk.back() * kMaxRestart * sizeof(double2)));
    L.ctrl.push_back(take(sizeof(Ctrl)));
    L.spec.push_back(o->pc == DIRAC_ST_PC_SPECTRAL ? take(spec_layout(&A[i]->prob, o->precision).total)
                     : line_kind(o->pc) ? take(line_layout(&A[i]->prob, o->precision, pc_slabs(o)).total)
                                                   : 0);
  }
  L.cap_rows = 0;
  L.cap_vec = 0;
  L.cap_lines = 0;
  for (int i = 0; i < nsys; i++) {
    L.cap_rows += spmv_wgs_cap(A[i]);
    L.cap_vec += L.nblk[i];
    if (line_kind(o->pc)) L.cap_lines += (line_layout(&A[i]->prob, o->precision, pc_slabs(o)).lines + 63) / 64;
  }
  L.tab_w = take(L.cap_rows * 2);
  L.tab_r = take(L.cap_rows * 2);
  L.tab_v = take(L.cap_vec * 2);
  L.tab_l = take(L.cap_lines * 2 + 2);
  L.desc = take(sizeof(BSys) * nsys);
  L.jobs = take(sizeof(LineJob) * nsys);
  L.sjobs = take(sizeof(LineSetupJob) * nsys);
  L.lists = take(sizeof(int64_t) * kListArrays * (nsys + 1));
  L.gather = take(sizeof(double) * 5 * nsys);
  L.total = off;
  return L;
}

// Device copies of the work lists of the current set of systems: active
// systems, then prefix sums of SpMV tiles (working lanes G), FP64-residual
// SpMV tiles, and 256-element vector blocks.
struct Lists {
  int64_t *dev = nullptr;
  int cap = 0;
  // workgroup tables and their capacities (entries)
  uint16_t *tab_w = nullptr, *tab_r = nullptr, *tab_v = nullptr, *tab_l = nullptr;
  int64_t cap_rows = 0, cap_vec = 0, cap_lines = 0;
  std::vector<int> cur;
  int G = -1, Gres = -1;
  WorkList w{}, r{}, v{}, ph[4]{};
  unsigned nw = 0, nr = 0, nv = 0, nph[4] = {0, 0, 0, 0};
  int64_t maxph[4] = {0, 0, 0, 0};  // largest per-system count of each phase
  std::vector<int64_t> host;

  int set(const std::vector<BSys> &hs, const std::vector<int> &act, int g, int gres, hipStream_t s) {
    if (act == cur && g == G && gres == Gres) return 0;
    cur = act;
    G = g;
    Gres = gres;
    const int na = (int)act.size();
    const size_t c1 = (size_t)cap + 1;
    host.assign(kListArrays * c1, 0);
    int64_t *ha = host.data(), *hw = ha + c1, *hr = hw + c1, *hv = hr + c1, *hp = hv + c1;
    for (int a = 0; a < na; a++) {
      const BSys &q = hs[act[a]];
      ha[a] = act[a];
      hw[a + 1] = hw[a] + spmv_wgs(q, g);
      hr[a + 1] = hr[a] + spmv_wgs(q, gres);
      hv[a + 1] = hv[a] + q.nblk;
      for (int k = 0; k < 4; k++) hp[k * c1 + a + 1] = hp[k * c1 + a] + q.lt[k];
    }
    for (int k = 0; k < 4; k++) {
      maxph[k] = 0;
      for (int a = 0; a < na; a++) maxph[k] = std::max(maxph[k], hs[act[a]].lt[k]);
    }
    bool fits = hw[na] < (int64_t(1) << 31) && hr[na] < (int64_t(1) << 31) && hv[na] < (int64_t(1) << 31);
    for (int k = 0; k < 4; k++) fits = fits && hp[k * c1 + na] < (int64_t(1) << 31);
    DST_CHECK(fits, "batch too large for one grid");
    // the workgroup tables are sized for the largest lane count
    DST_CHECK(hw[na] <= cap_rows && hr[na] <= cap_rows && hv[na] <= cap_vec && hp[3 * c1 + na] <= cap_lines,
              "internal: work list exceeds its table");
    nw = (unsigned)hw[na];
    nr = (unsigned)hr[na];
    nv = (unsigned)hv[na];
    w = {dev, dev + c1, tab_w, na};
    r = {dev, dev + 2 * c1, tab_r, na};
    v = {dev, dev + 3 * c1, tab_v, na};
    for (int k = 0; k < 4; k++) {
      nph[k] = (unsigned)hp[k * c1 + na];
      ph[k] = {dev, dev + (4 + k) * c1, k == 3 ? tab_l : nullptr, na};
    }
    DST_HIP(hipMemcpyAsync(dev, host.data(), host.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (na > 0) {
      g_fill_tab<<<na, 256, 0, s>>>(w.off, tab_w);
      g_fill_tab<<<na, 256, 0, s>>>(r.off, tab_r);
      g_fill_tab<<<na, 256, 0, s>>>(v.off, tab_v);
      if (cap_lines > 0) g_fill_tab<<<na, 256, 0, s>>>(ph[3].off, tab_l);
      DST_LAUNCHED();
    }
    // the host staging vector is rewritten by the next call: wait for the copy
    DST_HIP(hipStreamSynchronize(s));
    return 0;
  }
};

template <typename T, int NC, int MODE>
static hipError_t launch_g_spmv(int G, const BSys *S, const WorkList &L, unsigned nwg, int j,
                                hipStream_t s) {
  if (nwg == 0) return hipSuccess;
  if (NC == 2) {
    if (G == kLdsLanes) g_spmv<T, 2, kLdsLanes, MODE><<<nwg, 256, 0, s>>>(S, L, j);
    else if (G == 4) g_spmv<T, 2, 4, MODE><<<nwg, 256, 0, s>>>(S, L, j);
    else if (G == 8) g_spmv<T, 2, 8, MODE><<<nwg, 256, 0, s>>>(S, L, j);
    else if (G == 32) g_spmv<T, 2, 32, MODE><<<nwg, 256, 0, s>>>(S, L, j);
    else g_spmv<T, 2, 16, MODE><<<nwg, 256, 0, s>>>(S, L, j);
  } else {
    if (G == 32 && sizeof(T) == 4) g_spmv<T, 4, 32, MODE><<<nwg, 256, 0, s>>>(S, L, j);
    else g_spmv<T, 4, 64, MODE><<<nwg, 256, 0, s>>>(S, L, j);
  }
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_g_cgs(int mk, const BSys *S, const WorkList &L, unsigned nwg, int jp1,
                               hipStream_t s) {
  if (nwg == 0) return hipSuccess;
  switch (mk) {
    case 8: g_cgs<T, 8, MODE><<<nwg, 256, 0, s>>>(S, L, jp1); break;
    case 16: g_cgs<T, 16, MODE><<<nwg, 256, 0, s>>>(S, L, jp1); break;
    case 32: g_cgs<T, 32, MODE><<<nwg, 256, 0, s>>>(S, L, jp1); break;
    default:
      g_cgs<T, 64, MODE><<<nwg, 256, 0, s>>>(S, L, jp1);
      break;
  }
  return hipGetLastError();
}

// lanes per block row the SpMV may use, for (block size, precision)
static std::vector<int> lane_candidates(int nc, int prec) {
  if (nc == 2) return std::vector<int>{kLdsLanes, 4, 8, 16, 32};
  return prec == 32 ? std::vector<int>{32, 64} : std::vector<int>{64};
}

// autotune cache: (nc, precision, floor(log2 of the batch's block rows)) -> lanes
static std::mutex g_tune_mu;
static std::map<long, int> g_tune;
static int g_forced[2][2] = {{0, 0}, {0, 0}};  // [nc == 4][prec == 32]

static long tune_key(int nc, int prec, int64_t rows) {
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= rows) lg++;
  return (long)nc * 100000 + (long)prec * 100 + lg;
}

// Pick the SpMV lanes for a batch: a forced value, else the cache, else time
// every candidate on V_1 = A Z_0 over the whole batch (one warm-up launch and
// one timed launch each) and keep the fastest.
template <typename T>
static int choose_lanes(const std::vector<BSys> &hs, const BSys *dS, Lists &lists,
                        const std::vector<int> &all, int gres, int &G, hipStream_t s) {
  const int nc = hs[0].nc, prec = sizeof(T) == 8 ? 64 : 32;
  int64_t rows = 0;
  for (const BSys &q : hs) rows += q.nrows;
  const long key = tune_key(nc, prec, rows);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    G = g_forced[nc == 4][prec == 32];
    if (G) return 0;
    auto f = g_tune.find(key);
    if (f != g_tune.end()) {
      G = f->second;
      return 0;
    }
  }
  hipEvent_t e0, e1;
  DST_HIP(hipEventCreate(&e0));
  DST_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int rc = 0;
  for (int c : lane_candidates(nc, prec)) {
    if ((rc = lists.set(hs, all, c, gres, s))) break;
    g_zero<T><<<lists.nv, 256, 0, s>>>(dS, lists.v, 0);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && !rc; rep++) {
      hipError_t e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        e = nc == 2 ? launch_g_spmv<T, 2, 0>(c, dS, lists.w, lists.nw, 0, s)
                    : launch_g_spmv<T, 4, 0>(c, dS, lists.w, lists.nw, 0, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        set_error("SpMV autotuning failed: %s", hipGetErrorString(e));
        rc = DIRAC_ST_EHIP;
      }
    }
    if (!rc && ms < best) {
      best = ms;
      G = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = G;
  return 0;
}

static void fill_desc(BSys &q, const dirac_st_bsr *A) {
  q = BSys{};
  q.rp = A->row_ptr;
  q.ci = A->col_idx;
  q.val64 = A->val64;
  q.val32 = A->val32;
  q.bj64 = A->bjinv64;
  q.bj32 = A->bjinv32;
  q.nrows = A->nrows;
  q.n = A->nrows * A->nc;
  q.nblk = (q.n + 255) / 256;
  q.nc = A->nc;
  q.st = make_stencil(&A->prob);
}

template <typename T>
static int batched_impl(int nsys, const dirac_st_bsr *const *A, const void *const *b, void *const *x,
                        const dirac_st_opts *o, unsigned char *work, dirac_st_stats *stats,
                        hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const BatchLayout BL = batch_layout(nsys, A, o);
  const int m = o->restart;
  const int nc = A[0]->nc;
  std::vector<BSys> hs(nsys);
  std::vector<Precond> pcs(nsys);
  BSys *dS = (BSys *)(work + BL.desc);
  LineJob *dJ = (LineJob *)(work + BL.jobs);
  LineSetupJob *dSJ = (LineSetupJob *)(work + BL.sjobs);
  std::vector<LineJob> jobs(nsys);
  const bool linepc = line_kind(o->pc);
  std::vector<LineSetupJob> sjobs(linepc ? nsys : 0);
  std::vector<LineStaging> staging(linepc ? nsys : 0);
  double *dGat = (double *)(work + BL.gather);
  Lists lists;
  lists.dev = (int64_t *)(work + BL.lists);
  lists.cap = nsys;
  lists.tab_w = (uint16_t *)(work + BL.tab_w);
  lists.tab_r = (uint16_t *)(work + BL.tab_r);
  lists.tab_v = (uint16_t *)(work + BL.tab_v);
  lists.tab_l = (uint16_t *)(work + BL.tab_l);
  lists.cap_rows = BL.cap_rows;
  lists.cap_vec = BL.cap_vec;
  lists.cap_lines = BL.cap_lines;
  for (int i = 0; i < nsys; i++) {
    BSys &q = hs[i];
    fill_desc(q, A[i]);
    q.ldv = BL.ldv[i];
    q.V = work + BL.V[i];
    q.Z = work + BL.Z[i];
    q.r64 = (double2 *)(work + BL.r64[i]);
    q.x = (double2 *)x[i];
    q.b = (const double2 *)b[i];
    q.partial = (double2 *)(work + BL.partial[i]);
    q.ctrl = (Ctrl *)(work + BL.ctrl[i]);
    if (linepc) {
      // host part now; the factorisations run grouped once every system is prepared
      pcs[i].kind = o->pc;
      pcs[i].prec = sizeof(T) == 8 ? 64 : 32;
      pcs[i].A = A[i];
      pcs[i].slabs = pc_slabs(o);
      if (int rc = line_prepare<T>(pcs[i], A[i], work + BL.spec[i], staging[i], s)) return rc;
    } else if (o->pc != DIRAC_ST_PC_NONE) {
      const double vbar = o->vbar >= 0.0 ? o->vbar : 0.5 * A[i]->prob.v0;
      if (int rc = pc_setup<T>(pcs[i], A[i], o->pc, vbar, work + BL.spec[i], s)) return rc;
    }
    for (int k = 0; k < 4; k++) q.lt[k] = 0;
    if (linepc) {
      const LineLayout &LL = pcs[i].LL;
      const dirac_st_problem &pr = A[i]->prob;
      unsigned char *lb = pcs[i].line;
      const bool dbl = sizeof(T) == 8;
      LineJob &jb = jobs[i];
      jb = LineJob{};
      jb.Q = lb + (dbl ? LL.q64 : LL.q32);
      jb.W = lb + (dbl ? LL.w64 : LL.w32);
      jb.b1 = lb + LL.buf;
      jb.b2 = lb + LL.buf2;
      jb.fac = lb + LL.fac;
      jb.lined = lb + LL.lined;
      jb.pk = LL.pk;
      jb.pm = LL.pm;
      jb.d = pr.d;
      jb.nc = pr.nc;
      jb.nt = LL.tl;  // rows of one time slab; the time transform runs per slab
      jb.S = q.nrows / pr.n[0];
      jb.lines = LL.lines;
      for (int a = 0; a < 4; a++) jb.n[a] = a <= pr.d ? pr.n[a] : 1;
      const int64_t ncol = jb.S * pr.nc;
      q.lt[0] = (int64_t)LL.slabs * ((ncol + 63) / 64) * (LL.pm / 64);
      for (int a = 2; a <= pr.d; a++) {
        jb.F[a] = lb + (dbl ? LL.f64[a] : LL.f32[a]);
        jb.Fi[a] = lb + (dbl ? LL.fi64[a] : LL.fi32[a]);
        jb.dpk[a] = LL.dpk[a];
        jb.dpm[a] = LL.dpm[a];
        int64_t cols = pr.nc, batches = pr.n[0];
        for (int b = 1; b < a; b++) cols *= pr.n[b];
        for (int b = a + 1; b <= pr.d; b++) batches *= pr.n[b];
        q.lt[a - 1] = batches * ((cols + 63) / 64) * (LL.dpm[a] / 64);
      }
      q.lt[3] = (LL.lines + 63) / 64;
      LineSetupJob &sj = sjobs[i];
      sj.G = pcs[i].G;
      sj.tw = (const double2 *)(lb + LL.tw64);
      sj.lam = (const double2 *)(lb + LL.lam);
      sj.pot = (const double *)(lb + LL.pot);
      sj.fac = lb + LL.fac;
      sj.lined = lb + LL.lined;
      sj.lines = LL.lines;
      sj.flag = (int *)(lb + LL.flag);
    }
  }
  if (linepc) {
    DST_HIP(hipMemcpyAsync(dJ, jobs.data(), sizeof(LineJob) * nsys, hipMemcpyHostToDevice, s));
    DST_HIP(hipMemcpyAsync(dSJ, sjobs.data(), sizeof(LineSetupJob) * nsys, hipMemcpyHostToDevice, s));
  }
  auto upload_desc = [&]() -> int {
    DST_HIP(hipMemcpyAsync(dS, hs.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice, s));
    DST_HIP(hipStreamSynchronize(s));
    return 0;
  };
  if (int rc = upload_desc()) return rc;
  g_zero_ctrl<<<dim3(4, nsys), 256, 0, s>>>(dS);
  DST_LAUNCHED();

  std::vector<int> all(nsys);
  for (int i = 0; i < nsys; i++) all[i] = i;
  // FP64 residual SpMV lanes: the complex128 autotuned value once known
  int Gres = nc == 2 ? 32 : 64;
  int G = 0;
  if (int rc = choose_lanes<T>(hs, dS, lists, all, Gres, G, s)) return rc;
  if (sizeof(T) == 8) {
    Gres = G;
  } else {
    int64_t rows = 0;
    for (const BSys &q : hs) rows += q.nrows;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto f = g_tune.find(tune_key(nc, 64, rows));
    if (g_forced[nc == 4][0]) Gres = g_forced[nc == 4][0];
    else if (f != g_tune.end()) Gres = f->second;
  }

  for (int i = 0; i < nsys; i++) stats[i].est = 0.0;
  std::vector<double> bnorm(nsys, 0.0), relres(nsys, 1.0), rb(5 * (size_t)nsys);
  std::vector<int> its(nsys, 0), cycles(nsys, 0), conv(nsys, 0), broke(nsys, 0);
  // read-backs land in page-locked memory when it is available
  double *const pinned = (double *)readback_buffer(sizeof(double) * 5 * (size_t)nsys);
  auto gather = [&](int nact) -> int {
    g_gather<<<(nact + 63) / 64, 64, 0, s>>>(dS, lists.w.act, nact, dGat);
    DST_LAUNCHED();
    double *dst = pinned ? pinned : rb.data();
    DST_HIP(hipMemcpyAsync(dst, dGat, sizeof(double) * 5 * nact, hipMemcpyDeviceToHost, s));
    DST_HIP(hipStreamSynchronize(s));
    if (pinned) std::copy(pinned, pinned + 5 * (size_t)nact, rb.begin());
    return 0;
  };
  // norms of the listed systems into rb[5a + 4] (and ctrl->dots_norm2):
  // src 0: r64 = b - A x, then ||r64||; src 1: ||b||; src 2: ||x||
  auto norms = [&](int src) -> int {
    const unsigned na = (unsigned)lists.cur.size();
    if (src == 0) DST_HIP(nc == 2 ? (launch_g_spmv<double, 2, 1>(Gres, dS, lists.r, lists.nr, 0, s))
                                  : (launch_g_spmv<double, 4, 1>(Gres, dS, lists.r, lists.nr, 0, s)));
    g_norm<<<lists.nv, 256, 0, s>>>(dS, lists.v, src);
    g_reduce<<<dim3(1, na), 256, 0, s>>>(dS, lists.w.act, 1, 0);
    DST_LAUNCHED();
    return gather((int)na);
  };

  if (int rc = lists.set(hs, all, G, Gres, s)) return rc;
  if (linepc) {
    const int d = A[0]->prob.d;
    if (d == 1) g_line_setup<T, 2, 1><<<lists.nph[3], 64, 0, s>>>(dSJ, lists.ph[3]);
    else if (d == 2) g_line_setup<T, 2, 2><<<lists.nph[3], 64, 0, s>>>(dSJ, lists.ph[3]);
    else g_line_setup<T, 4, 3><<<lists.nph[3], 64, 0, s>>>(dSJ, lists.ph[3]);
    DST_LAUNCHED();
    std::vector<int> bad(nsys, 0);
    static_assert(sizeof(int) <= 5 * sizeof(double), "flags fit the gather area");
    g_line_flags<<<(nsys + 63) / 64, 64, 0, s>>>(dSJ, nsys, (int *)dGat);
    DST_LAUNCHED();
    int *fdst = pinned ? (int *)pinned : bad.data();
    DST_HIP(hipMemcpyAsync(fdst, dGat, sizeof(int) * nsys, hipMemcpyDeviceToHost, s));
    DST_HIP(hipStreamSynchronize(s));
    if (pinned) std::copy((int *)pinned, (int *)pinned + nsys, bad.begin());
    for (int i = 0; i < nsys; i++)
      DST_CHECK(bad[i] == 0, "system %d: line preconditioner has %d singular line factorisations", i, bad[i]);
    staging.clear();
  }
  // a zero initial guess needs no first SpMV: its residual is b.  The norm
  // of b is taken last so that ctrl->dots_norm2 holds ||b||^2 afterwards.
  if (int rc = norms(2)) return rc;
  std::vector<char> xzero(nsys);
  for (int i = 0; i < nsys; i++) xzero[i] = rb[5 * i + 4] == 0.0;
  if (int rc = norms(1)) return rc;
  std::vector<int> active, zero_b;
  for (int i = 0; i < nsys; i++) {
    bnorm[i] = sqrt(rb[5 * i + 4]);
    if (!std::isfinite(bnorm[i])) broke[i] = 1;
    else if (bnorm[i] == 0.0) zero_b.push_back(i);
    else active.push_back(i);
  }
  if (!zero_b.empty()) {  // b = 0: x = 0 solves the system exactly
    if (int rc = lists.set(hs, zero_b, G, Gres, s)) return rc;
    g_zero<T><<<lists.nv, 256, 0, s>>>(dS, lists.v, 1);
    DST_LAUNCHED();
    for (int i : zero_b) {
      conv[i] = 1;
      relres[i] = 0.0;
    }
  }

  std::vector<double> sigma(nsys, 1.0), rstart(nsys, 0.0);
  bool first = true;
  while (!active.empty()) {
    // FP64 true residuals decide convergence and restart
    if (int rc = lists.set(hs, active, G, Gres, s)) return rc;
    bool all_zero = first;
    for (int i : active) all_zero = all_zero && xzero[i];
    if (all_zero) {
      g_copy_b<<<lists.nv, 256, 0, s>>>(dS, lists.v);
      DST_LAUNCHED();
      for (size_t a = 0; a < active.size(); a++) rb[5 * a + 4] = bnorm[active[a]] * bnorm[active[a]];
    } else if (int rc = norms(0)) {
      return rc;
    }
    first = false;
    std::vector<int> cyc;
    for (size_t a = 0; a < active.size(); a++) {
      const int i = active[a];
      const double rn = sqrt(rb[5 * a + 4]);
      relres[i] = rn / bnorm[i];
      rstart[i] = rn;
      if (!std::isfinite(rn)) broke[i] = 1;
      else if (relres[i] <= o->rtol) conv[i] = 1;
      else if (its[i] < o->max_it && (o->max_cycles <= 0 || cycles[i] < o->max_cycles)) cyc.push_back(i);
    }
    active = cyc;
    if (active.empty()) break;
    // start the cycle: V_0 = r / ||r||, g = ||r|| e_1, sigma_0 = 1
    if (int rc = lists.set(hs, active, G, Gres, s)) return rc;
    g_v0<T><<<lists.nv, 256, 0, s>>>(dS, lists.v);
    g_cycle_init<<<(unsigned)active.size(), 64, 0, s>>>(dS, lists.w.act);
    DST_LAUNCHED();
    for (int i : active) {
      cycles[i]++;
      sigma[i] = 1.0;
      hs[i].k = 0;
    }
    std::vector<int> step = active;
    for (int j = 0; j < m && !step.empty(); j++) {
      if (int rc = lists.set(hs, step, G, Gres, s)) return rc;
      const unsigned na = (unsigned)step.size();
      // Z_j = M^{-1} (sigma_j V_j)
      if (linepc) {
        // Q along time, transverse DFTs, line solves, inverse DFTs, sigma_j W
        const int d = A[0]->prob.d;
        const int64_t *act = lists.w.act;
        auto grid = [&](int k) { return dim3((unsigned)lists.maxph[k], na); };
        launch_line_gemm<T>(0, false, 0, 1, grid(0), dS, dJ, act, j, s);
        int cur = 1, oth = 2;
        for (int a = d; a >= 2; a--) {
          launch_line_gemm<T>(a, false, cur, oth, grid(a - 1), dS, dJ, act, j, s);
          std::swap(cur, oth);
        }
        if (nc == 2) g_line_solve<T, 2><<<lists.nph[3], 64, 0, s>>>(dJ, lists.ph[3], cur);
        else g_line_solve<T, 4><<<lists.nph[3], 64, 0, s>>>(dJ, lists.ph[3], cur);
        for (int a = 2; a <= d; a++) {
          launch_line_gemm<T>(a, true, cur, oth, grid(a - 1), dS, dJ, act, j, s);
          std::swap(cur, oth);
        }
        launch_line_gemm<T>(0, false, cur, 3, grid(0), dS, dJ, act, j, s);
      } else if (o->pc == DIRAC_ST_PC_SPECTRAL) {
        for (int i : step) {
          const cx<T> *vj = (const cx<T> *)hs[i].V + (int64_t)j * hs[i].ldv;
          cx<T> *zj = (cx<T> *)hs[i].Z + (int64_t)j * hs[i].ldv;
          if (int rc = pc_apply_base<T>(pcs[i], vj, zj, sigma[i], hs[i].n, s)) return rc;
        }
      } else if (o->pc == DIRAC_ST_PC_BLOCK_JACOBI) {
        if (nc == 2) g_pc_local<T, 2, true><<<lists.nv, 256, 0, s>>>(dS, lists.v, j);
        else g_pc_local<T, 4, true><<<lists.nv, 256, 0, s>>>(dS, lists.v, j);
      } else {
        g_pc_local<T, 2, false><<<lists.nv, 256, 0, s>>>(dS, lists.v, j);
      }
      DST_LAUNCHED();
      // V_{j+1} = A Z_j
      DST_HIP(nc == 2 ? (launch_g_spmv<T, 2, 0>(G, dS, lists.w, lists.nw, j, s))
                      : (launch_g_spmv<T, 4, 0>(G, dS, lists.w, lists.nw, j, s)));
      // two classical Gram-Schmidt passes and the norm, as in the single solver
      const int jp1 = j + 1;
      const int mk = jp1 <= 8 ? 8 : jp1 <= 16 ? 16 : jp1 <= 32 ? 32 : 64;
      DST_HIP((launch_g_cgs<T, DOTS>(mk, dS, lists.v, lists.nv, jp1, s)));
      g_reduce<<<dim3(jp1, na), 256, 0, s>>>(dS, lists.w.act, 0, 1);
      DST_LAUNCHED();
      DST_HIP((launch_g_cgs<T, UPDOTS>(mk, dS, lists.v, lists.nv, jp1, s)));
      g_reduce<<<dim3(jp1, na), 256, 0, s>>>(dS, lists.w.act, 0, 2);
      DST_LAUNCHED();
      DST_HIP((launch_g_cgs<T, UPNORM>(mk, dS, lists.v, lists.nv, jp1, s)));
      g_reduce<<<dim3(1, na), 256, 0, s>>>(dS, lists.w.act, 1, 0);
      g_givens<<<na, 64, 0, s>>>(dS, lists.w.act, j);
      DST_LAUNCHED();
      if (int rc = gather((int)na)) return rc;
      std::vector<int> next;
      for (size_t a = 0; a < step.size(); a++) {
        const int i = step[a];
        its[i]++;
        hs[i].k = j + 1;
        const double est_abs = rb[5 * a], happy = rb[5 * a + 1], fin = rb[5 * a + 2];
        sigma[i] = rb[5 * a + 3];
        stats[i].est = est_abs / bnorm[i];
        if (fin == 0.0 || !std::isfinite(est_abs)) {
          broke[i] = 1;
          continue;
        }
        if (stats[i].est <= o->rtol || happy != 0.0 || its[i] >= o->max_it) continue;
        if (sizeof(T) == 4 && o->inner_rtol > 0.0 && est_abs <= o->inner_rtol * rstart[i]) continue;
        next.push_back(i);
      }
      step = next;
    }
    // x += Z y for every system of the cycle that did not break down
    std::vector<int> upd;
    for (int i : active)
      if (!broke[i]) upd.push_back(i);
    active = upd;
    if (active.empty()) break;
    if (int rc = upload_desc()) return rc;  // carries the step counts k
    if (int rc = lists.set(hs, active, G, Gres, s)) return rc;
    g_backsub<<<(unsigned)active.size(), 64, 0, s>>>(dS, lists.w.act);
    g_update<T><<<lists.nv, 256, 0, s>>>(dS, lists.v);
    DST_LAUNCHED();
  }
  DST_HIP(hipStreamSynchronize(s));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  int rc = DIRAC_ST_OK;
  for (int i = 0; i < nsys; i++) {
    stats[i].iters = its[i];
    stats[i].cycles = cycles[i];
    stats[i].converged = conv[i];
    stats[i].singular_blocks = A[i]->singular_blocks;
    stats[i].relres = relres[i];
    stats[i].ms = ms;
    stats[i].fallback = 0;
    if (broke[i]) rc = DIRAC_ST_EBREAKDOWN;
    else if (!conv[i] && rc == DIRAC_ST_OK) rc = DIRAC_ST_NOT_CONVERGED;
  }
  if (rc == DIRAC_ST_EBREAKDOWN) set_error("NaN or Inf in at least one system of the batch");
  return rc;
}

}  // namespace dst

using namespace dst;

static int check_batch(int32_t nsys, const dirac_st_bsr *const *A) {
  DST_CHECK(nsys >= 1 && nsys <= kMaxBatch && A, "batch size must be in 1..%d", kMaxBatch);
  for (int i = 0; i < nsys; i++) {
    DST_CHECK(A[i] && A[i]->row_ptr && A[i]->col_idx && A[i]->val64, "system %d: matrix arrays are NULL", i);
    DST_CHECK(A[i]->nrows >= 1, "system %d: empty matrix", i);
    DST_CHECK(A[i]->nc == A[0]->nc, "all systems of a batch must have the same block size");
  }
  return 0;
}

static int check_batch_opts(int32_t nsys, const dirac_st_bsr *const *A, const dirac_st_opts *o) {
  if (int rc = check_batch(nsys, A)) return rc;
  DST_CHECK(o, "opts is NULL");
  DST_CHECK(o->restart >= 1 && o->restart <= kMaxRestart, "restart must be in 1..%d", kMaxRestart);
  DST_CHECK(o->precision == 64 || o->precision == 32, "precision must be 64 or 32");
  DST_CHECK(o->rtol > 0.0 && o->max_it >= 0, "rtol must be positive and max_it >= 0");
  DST_CHECK(o->matrix_free == 0, "the batched solver applies the stored blocks (matrix_free must be 0)");
  for (int i = 0; i < nsys; i++) {
    if (int rc = check_pc_opts(A[i], o)) return rc;
    DST_CHECK(A[i]->prob.d == A[0]->prob.d, "all systems of a batched solve must have the same dimension");
    DST_CHECK(o->precision == 64 || A[i]->val32, "system %d: precision 32 needs val32", i);
    if (o->pc == DIRAC_ST_PC_BLOCK_JACOBI)
      DST_CHECK(o->precision == 64 ? A[i]->bjinv64 != nullptr : A[i]->bjinv32 != nullptr,
                "system %d: block-Jacobi preconditioner needs bjinv%d", i, o->precision);
  }
  return 0;
}

extern "C" size_t dirac_st_batched_workspace_bytes(int32_t nsys, const dirac_st_bsr *const *A,
                                                   const dirac_st_opts *opts) {
  clear_error();
  if (check_batch_opts(nsys, A, opts)) return 0;
  return batch_layout(nsys, A, opts).total;
}

extern "C" int dirac_st_fgmres_batched(int32_t nsys, const dirac_st_bsr *const *A,
                                       const void *const *b, void *const *x,
                                       const dirac_st_opts *opts, void *work, size_t work_bytes,
                                       dirac_st_stats *stats, void *stream) {
  clear_error();
  if (int rc = check_batch_opts(nsys, A, opts)) return rc;
  DST_CHECK(b && x && work && stats, "b, x, work and stats must be set");
  for (int i = 0; i < nsys; i++) DST_CHECK(b[i] && x[i], "system %d: b or x is NULL", i);
  const size_t need = batch_layout(nsys, A, opts).total;
  if (work_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", work_bytes, need);
    return DIRAC_ST_ENOSPACE;
  }
  DST_CHECK(((uintptr_t)work & 255) == 0, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (opts->precision == 64)
    return batched_impl<double>(nsys, A, b, x, opts, (unsigned char *)work, stats, s);
  return batched_impl<float>(nsys, A, b, x, opts, (unsigned char *)work, stats, s);
}

// Workspace of dirac_st_spmv_batched: descriptors, list arrays, workgroup
// tables (sized for the largest lane count).
struct SpmvBatchLayout {
  size_t desc, lists, tab_w, tab_r, tab_v, total;
  int64_t cap_rows, cap_vec;
};

static SpmvBatchLayout spmv_batch_layout(int32_t nsys, const dirac_st_bsr *const *A) {
  SpmvBatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t r = off;
    off += align256(b);
    return r;
  };
  for (int i = 0; i < nsys; i++) {
    L.cap_rows += spmv_wgs_cap(A[i]);
    L.cap_vec += (A[i]->nrows * A[i]->nc + 255) / 256;
  }
  L.desc = take(sizeof(BSys) * nsys);
  L.lists = take(sizeof(int64_t) * kListArrays * (nsys + 1));
  L.tab_w = take(L.cap_rows * 2);
  L.tab_r = take(L.cap_rows * 2);
  L.tab_v = take(L.cap_vec * 2);
  L.total = off;
  return L;
}

extern "C" size_t dirac_st_spmv_batched_workspace_bytes(int32_t nsys, const dirac_st_bsr *const *A) {
  clear_error();
  if (check_batch(nsys, A)) return 0;
  return spmv_batch_layout(nsys, A).total;
}

extern "C" int dirac_st_spmv_batched(int32_t nsys, const dirac_st_bsr *const *A, int32_t prec,
                                     const void *const *x, void *const *y, int32_t lanes, void *work,
                                     size_t work_bytes, void *stream) {
  clear_error();
  if (int rc = check_batch(nsys, A)) return rc;
  DST_CHECK(prec == 64 || prec == 32, "precision must be 64 or 32");
  DST_CHECK(x && y && work, "x, y and work must be set");
  const int nc = A[0]->nc;
  const std::vector<int> cands = lane_candidates(nc, prec);
  DST_CHECK(std::find(cands.begin(), cands.end(), (int)lanes) != cands.end(),
            "lanes %d not available for %dx%d blocks at precision %d", lanes, nc, nc, prec);
  const SpmvBatchLayout SL = spmv_batch_layout(nsys, A);
  if (work_bytes < SL.total) {
    set_error("workspace too small: %zu < %zu bytes", work_bytes, SL.total);
    return DIRAC_ST_ENOSPACE;
  }
  DST_CHECK(((uintptr_t)work & 255) == 0, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  std::vector<BSys> hs(nsys);
  for (int i = 0; i < nsys; i++) {
    DST_CHECK(x[i] && y[i], "system %d: x or y is NULL", i);
    DST_CHECK(prec == 64 || A[i]->val32, "system %d: precision 32 needs val32", i);
    fill_desc(hs[i], A[i]);
    hs[i].Z = const_cast<void *>(x[i]);  // V_{j+1} = A Z_j with j = 0 and ldv = 0: y = A x
    hs[i].V = y[i];
    hs[i].ldv = 0;
  }
  unsigned char *wb = (unsigned char *)work;
  BSys *dS = (BSys *)(wb + SL.desc);
  Lists lists;
  lists.dev = (int64_t *)(wb + SL.lists);
  lists.cap = nsys;
  lists.tab_w = (uint16_t *)(wb + SL.tab_w);
  lists.tab_r = (uint16_t *)(wb + SL.tab_r);
  lists.tab_v = (uint16_t *)(wb + SL.tab_v);
  lists.cap_rows = SL.cap_rows;
  lists.cap_vec = SL.cap_vec;
  DST_HIP(hipMemcpyAsync(dS, hs.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice, s));
  std::vector<int> all(nsys);
  for (int i = 0; i < nsys; i++) all[i] = i;
  if (int rc = lists.set(hs, all, lanes, nc == 2 ? 32 : 64, s)) return rc;  // synchronises
  if (prec == 64)
    DST_HIP(nc == 2 ? (launch_g_spmv<double, 2, 0>(lanes, dS, lists.w, lists.nw, 0, s))
                    : (launch_g_spmv<double, 4, 0>(lanes, dS, lists.w, lists.nw, 0, s)));
  else
    DST_HIP(nc == 2 ? (launch_g_spmv<float, 2, 0>(lanes, dS, lists.w, lists.nw, 0, s))
                    : (launch_g_spmv<float, 4, 0>(lanes, dS, lists.w, lists.nw, 0, s)));
  return 0;
}

extern "C" int dirac_st_batched_set_lanes(int32_t nc, int32_t prec, int32_t lanes) {
  clear_error();
  DST_CHECK((nc == 2 || nc == 4) && (prec == 64 || prec == 32), "nc must be 2 or 4, prec 64 or 32");
  const std::vector<int> cands = lane_candidates(nc, prec);
  DST_CHECK(lanes == 0 || std::find(cands.begin(), cands.end(), (int)lanes) != cands.end(),
            "lanes %d not available for %dx%d blocks at precision %d", lanes, nc, nc, prec);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_forced[nc == 4][prec == 32] = lanes;
  return 0;
}

extern "C" int32_t dirac_st_batched_lanes(int32_t nc, int32_t prec, int64_t rows) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int f = (nc == 2 || nc == 4) && (prec == 64 || prec == 32) ? g_forced[nc == 4][prec == 32] : 0;
  if (f) return f;
  auto it = g_tune.find(tune_key(nc, prec, rows));
  return it == g_tune.end() ? 0 : it->second;
}
