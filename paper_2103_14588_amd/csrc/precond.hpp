// precond.hpp -- the base preconditioners M of right-preconditioned GMRES
// (Sec. 2.2): node-block Jacobi (inverses of the diagonal nc x nc blocks),
// the spatial-Fourier preconditioner (the operator with the potential replaced
// by a constant, inverted exactly: DFT over every periodic spatial axis, one
// block-tridiagonal solve in time per Fourier mode, inverse DFT) and the line
// preconditioner (exact inverse for potentials that depend on x only: time
// eigenbasis, DFT over the transverse axes, periodic block-tridiagonal solves
// along x).
#pragma once

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "common.hpp"
#include "krylov.hpp"
#include "linepc.hpp"
#include "readback.hpp"
#include "spectral.hpp"
#include "time_eigen.hpp"

namespace dst {

static inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// the line and time-slab preconditioners share their set-up and apply
static inline bool line_kind(int pc) { return pc == DIRAC_ST_PC_LINE || pc == DIRAC_ST_PC_TIME_SLABS; }
static inline int pc_slabs(const dirac_st_opts *o) { return o->pc == DIRAC_ST_PC_TIME_SLABS ? o->time_slabs : 1; }

// preconditioner parameters that the problem must admit
static inline int check_pc_opts(const dirac_st_bsr *A, const dirac_st_opts *o) {
  DST_CHECK(o->pc >= DIRAC_ST_PC_NONE && o->pc <= DIRAC_ST_PC_TIME_SLABS, "unknown preconditioner %d", o->pc);
  if (o->pc == DIRAC_ST_PC_TIME_SLABS)
    DST_CHECK(o->time_slabs >= 1 && A->prob.n[0] % o->time_slabs == 0,
              "time_slabs must be >= 1 and divide n_t = %d (got %d)", A->prob.n[0], o->time_slabs);
  return 0;
}

// ------------------------------------------------------------ preconditioner
struct Precond {
  int kind = DIRAC_ST_PC_NONE;
  int prec = 64;
  const dirac_st_bsr *A = nullptr;
  // spectral
  SpecGeom G{};
  unsigned char *spec = nullptr;
  SpecLayout SL{};
  // line (shares G and the twiddle tables' geometry)
  unsigned char *line = nullptr;
  LineLayout LL{};
  int slabs = 1;  // time slabs of DIRAC_ST_PC_TIME_SLABS (1 for the line preconditioner)
  // learned correction z += s N(v / s) (flexible GMRES only)
  const dirac_st_nn *nn = nullptr;
  bool nn_on = false;
  unsigned char *nnwork = nullptr;
  // spectral: the pivot inverses are computed by the first application after
  // the set-up (inside its block elimination) rather than by a pass of their own
  mutable bool piv_pending = false;
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
  gamma_set(p->d, G.g);
}

// Twiddles exp(-2 pi i q / n_a) of every spatial axis, FP64 and FP32 copies,
// computed on the device (no host staging, no synchronisation).
static __global__ void twiddle_kernel(SpecGeom G, double2 *__restrict__ tw64, float2 *__restrict__ tw32) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  for (int a = 1; a <= G.d; a++) {
    if (q >= G.n[a]) continue;
    double sn, cs;
    sincospi(2.0 * (double)q / (double)G.n[a], &sn, &cs);
    tw64[G.tw_off[a] + q] = mk<double2>(cs, -sn);
    tw32[G.tw_off[a] + q] = mk<float2>((float)cs, (float)-sn);
  }
}

static int spec_twiddles(const SpecGeom &G, unsigned char *base, const SpecLayout &L, hipStream_t s) {
  int nmax = 1;
  for (int a = 1; a <= G.d; a++) nmax = G.n[a] > nmax ? G.n[a] : nmax;
  twiddle_kernel<<<(nmax + 255) / 256, 256, 0, s>>>(G, (double2 *)(base + L.tw64), (float2 *)(base + L.tw32));
  DST_LAUNCHED();
  return 0;
}

// Line preconditioner set-up: time eigen-decomposition and 1D potential
// matrix on the host (FP64), per-line factors on the device.
static double host_potential(const dirac_st_problem *p, double x) {
  if (p->vkind == DIRAC_ST_V_STEP) return x > p->x0 ? p->v0 : 0.0;
  if (p->vkind == DIRAC_ST_V_SMOOTH) return 0.5 * p->v0 * (1.0 + tanh((x - p->x0) / p->lw));
  return 0.0;
}

// Host tables of the line preconditioner for one (problem, precision, time
// slabs): twiddles, time eigen-decomposition, 1D potential matrix and the
// transverse DFT matrices, packed in one page-locked block together with each
// piece's offset in the workspace.  They depend on nothing else, so a set-up
// of a problem seen before only uploads them (asynchronously: copies from
// page-locked memory do not stage through the driver).
struct LineTables {
  struct Piece {
    size_t dev, host, bytes;
  };
  std::vector<Piece> pieces;
  unsigned char *host = nullptr;
  bool pinned = false;
  LineTables() = default;
  LineTables(const LineTables &) = delete;
  LineTables &operator=(const LineTables &) = delete;
  ~LineTables() {
    if (!host) return;
    if (pinned) (void)hipHostFree(host);
    else delete[] host;
  }
};

// Host-side data of one line preconditioner set-up; kept alive until the
// stream has consumed the asynchronous copies made from it.
struct LineStaging {
  std::shared_ptr<const LineTables> tables;
};

static int build_line_tables(const dirac_st_problem *p, const LineLayout &L, const SpecGeom &G,
                             std::shared_ptr<LineTables> &out) {
  std::vector<std::pair<size_t, std::vector<unsigned char>>> parts;  // (workspace offset, bytes)
  auto add = [&](size_t off, const void *src, size_t bytes) {
    const unsigned char *c = (const unsigned char *)src;
    parts.emplace_back(off, std::vector<unsigned char>(c, c + bytes));
  };
  int64_t twn = 0;
  for (int a = 1; a <= p->d; a++) twn += p->n[a];
  std::vector<double2> tw64(twn, mk<double2>(0, 0));
  std::vector<float2> tw32(twn, mk<float2>(0, 0));
  for (int a = 1; a <= p->d; a++)
    for (int q = 0; q < p->n[a]; q++) {
      const double th = 2.0 * M_PI * (double)q / (double)p->n[a];
      tw64[G.tw_off[a] + q] = mk<double2>(cos(th), -sin(th));
      tw32[G.tw_off[a] + q] = mk<float2>((float)cos(th), (float)-sin(th));
    }
  add(L.tw64, tw64.data(), twn * sizeof(double2));
  add(L.tw32, tw32.data(), twn * sizeof(float2));
  // every slab has the pencil of a whole interval of tl rows (first row
  // interior-like, last row the end row), so one decomposition serves all
  const int nt = p->n[0], n1 = p->n[1], tl = L.tl;
  std::vector<std::complex<double>> lam, W, Q;
  if (int rc = time_eigen(tl, p->len[0] / nt, lam, W, Q)) return rc;
  std::vector<double2> q64((size_t)L.pm * L.pk, mk<double2>(0, 0)), w64 = q64;
  std::vector<float2> q32(q64.size(), mk<float2>(0, 0)), w32 = q32;
  std::vector<double2> l64(nt);  // eigenvalue of time row r: that of its row in the slab
  for (int r = 0; r < nt; r++) l64[r] = mk<double2>(lam[r % tl].real(), lam[r % tl].imag());
  for (int r = 0; r < tl; r++)
    for (int c = 0; c < tl; c++) {
      const size_t e = (size_t)r * L.pk + c;
      const std::complex<double> qv = Q[(size_t)r * tl + c], wv = W[(size_t)r * tl + c];
      q64[e] = mk<double2>(qv.real(), qv.imag());
      w64[e] = mk<double2>(wv.real(), wv.imag());
      q32[e] = mk<float2>((float)qv.real(), (float)qv.imag());
      w32[e] = mk<float2>((float)wv.real(), (float)wv.imag());
    }
  add(L.lam, l64.data(), l64.size() * sizeof(double2));
  add(L.q64, q64.data(), q64.size() * sizeof(double2));
  add(L.w64, w64.data(), w64.size() * sizeof(double2));
  add(L.q32, q32.data(), q32.size() * sizeof(float2));
  add(L.w32, w32.data(), w32.size() * sizeof(float2));
  // P_x: diagonal and (i, i+1) entries, 2-point Gauss on every element
  std::vector<double> pot(2 * (size_t)n1, 0.0);
  const double h1 = p->len[1] / n1, r3 = 0.57735026918962576451;
  for (int e = 0; e < n1; e++)
    for (int q = 0; q < 2; q++) {
      const double xi = 0.5 * (1.0 + (q ? r3 : -r3));
      const double w = 0.5 * h1 * host_potential(p, (e + xi) * h1);
      pot[e] += w * (1.0 - xi) * (1.0 - xi);
      pot[(e + 1) % n1] += w * xi * xi;
      pot[n1 + e] += w * (1.0 - xi) * xi;
    }
  add(L.pot, pot.data(), pot.size() * sizeof(double));
  // DFT matrices of the transverse axes: F[k][j] = exp(-2 pi i k j / n),
  // F^{-1}[j][k] = exp(2 pi i j k / n) / n
  for (int a = 2; a <= p->d; a++) {
    const int n = p->n[a], pk = L.dpk[a];
    const size_t e = (size_t)L.dpm[a] * pk;
    std::vector<double2> f64(e, mk<double2>(0, 0)), fi64 = f64;
    std::vector<float2> f32(e, mk<float2>(0, 0)), fi32 = f32;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++) {
        const double th = 2.0 * M_PI * (double)((int64_t)k * j % n) / n;
        const double c = cos(th), sn = sin(th);
        f64[(size_t)k * pk + j] = mk<double2>(c, -sn);
        fi64[(size_t)k * pk + j] = mk<double2>(c / n, sn / n);
        f32[(size_t)k * pk + j] = mk<float2>((float)c, (float)-sn);
        fi32[(size_t)k * pk + j] = mk<float2>((float)(c / n), (float)(sn / n));
      }
    add(L.f64[a], f64.data(), e * 16);
    add(L.fi64[a], fi64.data(), e * 16);
    add(L.f32[a], f32.data(), e * 8);
    add(L.fi32[a], fi32.data(), e * 8);
  }
  // the pieces fill two contiguous ranges of the workspace layout, the
  // tables before the factors [0, fac) and the DFT matrices [f64[2], total):
  // the host block is an image of both, uploaded in (at most) two copies
  const size_t r1 = L.fac, r2b = p->d >= 2 ? L.f64[2] : L.total, r2 = L.total - r2b;
  auto T = std::make_shared<LineTables>();
  const size_t total = r1 + r2;
  if (hipHostMalloc((void **)&T->host, total, hipHostMallocDefault) == hipSuccess) {
    T->pinned = true;
  } else {
    (void)hipGetLastError();  // handled: the tables live in pageable memory instead
    T->host = new unsigned char[total];
  }
  memset(T->host, 0, total);
  for (auto &pt : parts) {
    const size_t at = pt.first < r1 ? pt.first : r1 + (pt.first - r2b);
    DST_CHECK(pt.first + pt.second.size() <= (pt.first < r1 ? r1 : L.total) && (pt.first < r1 || pt.first >= r2b),
              "line preconditioner table outside its workspace range");
    memcpy(T->host + at, pt.second.data(), pt.second.size());
  }
  T->pieces.push_back({0, 0, r1});
  if (r2 > 0) T->pieces.push_back({r2b, r1, r2});
  out = std::move(T);
  return 0;
}

// Cached tables of (problem, precision, slabs); at most kLineTableCache
// entries are kept (a set-up in flight holds its own reference).  The cache
// is never destroyed: freeing page-locked memory from a static destructor
// could run after the HIP runtime has shut down.
constexpr size_t kLineTableCache = 256;
static int line_tables(const dirac_st_problem *p, int prec, const LineLayout &L, const SpecGeom &G,
                       std::shared_ptr<const LineTables> &out) {
  static std::mutex &mu = *new std::mutex;
  static auto &cache = *new std::map<std::vector<double>, std::shared_ptr<const LineTables>>;
  std::vector<double> key = {(double)p->d, (double)p->nc, (double)p->vkind, p->m, p->v0, p->x0, p->lw,
                             (double)prec, (double)L.slabs};
  for (int a = 0; a < 4; a++) {
    key.push_back((double)p->n[a]);
    key.push_back(p->len[a]);
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    auto f = cache.find(key);
    if (f != cache.end()) {
      out = f->second;
      return 0;
    }
  }
  std::shared_ptr<LineTables> built;
  if (int rc = build_line_tables(p, L, G, built)) return rc;
  std::lock_guard<std::mutex> lk(mu);
  if (cache.size() >= kLineTableCache) cache.clear();
  cache[key] = built;
  out = built;
  return 0;
}

// Geometry, time eigen-decomposition, 1D potential matrix, DFT matrices:
// computed on the host (once per problem) and copied asynchronously into the
// workspace; the failure flag is cleared.  The factorisation itself is
// line_factor.
template <typename T>
static int line_prepare(Precond &P, const dirac_st_bsr *A, unsigned char *base, LineStaging &st,
                        hipStream_t s) {
  const dirac_st_problem *p = &A->prob;
  DST_CHECK(P.slabs >= 1 && p->n[0] % P.slabs == 0, "time slabs must divide n_t");
  DST_CHECK(p->n[0] / P.slabs <= kTimeEigenMax, "line preconditioner needs n_t per slab <= %d", kTimeEigenMax);
  P.line = base;
  P.LL = line_layout(p, P.prec, P.slabs);
  const LineLayout &L = P.LL;
  spec_geom(p, 0.0, P.G);
  if (int rc = line_tables(p, P.prec, L, P.G, st.tables)) return rc;
  for (const LineTables::Piece &pc : st.tables->pieces)
    DST_HIP(hipMemcpyAsync(base + pc.dev, st.tables->host + pc.host, pc.bytes, hipMemcpyHostToDevice, s));
  zero_i32_flag<<<1, 64, 0, s>>>((int *)(base + L.flag));
  DST_LAUNCHED();
  return 0;
}

// Per-line factorisation of one operator (after line_prepare).
template <typename T>
static int line_factor(const Precond &P, hipStream_t s) {
  const LineLayout &L = P.LL;
  unsigned char *base = P.line;
  const unsigned g = (unsigned)((L.lines + 63) / 64);
  const double2 *tw64 = (const double2 *)(base + L.tw64);
  const double2 *lamd = (const double2 *)(base + L.lam);
  const double *potd = (const double *)(base + L.pot);
  cx<T> *fac = (cx<T> *)(base + L.fac), *lined = (cx<T> *)(base + L.lined);
  int *flag = (int *)(base + L.flag);
  if (P.G.d == 1)
    line_setup<T, 2, 1><<<g, 64, 0, s>>>(P.G, tw64, lamd, potd, fac, lined, L.lines, flag);
  else if (P.G.d == 2)
    line_setup<T, 2, 2><<<g, 64, 0, s>>>(P.G, tw64, lamd, potd, fac, lined, L.lines, flag);
  else
    line_setup<T, 4, 3><<<g, 64, 0, s>>>(P.G, tw64, lamd, potd, fac, lined, L.lines, flag);
  DST_LAUNCHED();
  return 0;
}

// Line preconditioner set-up of one operator: prepare, factorise, check the
// failure flag (synchronises the stream).
template <typename T>
static int line_setup_host(Precond &P, const dirac_st_bsr *A, unsigned char *base, hipStream_t s) {
  LineStaging st;
  if (int rc = line_prepare<T>(P, A, base, st, s)) return rc;
  if (int rc = line_factor<T>(P, s)) return rc;
  int local = 0;
  int *const pinned = (int *)readback_buffer(sizeof(int));
  int *const bad = pinned ? pinned : &local;
  DST_HIP(hipMemcpyAsync(bad, base + P.LL.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  // the staging holds the uploaded tables: wait for every copy
  DST_HIP(hipStreamSynchronize(s));
  DST_CHECK(*bad == 0, "line preconditioner: %d singular or non-finite line factorisations", *bad);
  return 0;
}

// One DFT pass along spatial axis a over a vector with `stride` elements
// between consecutive nodes of that axis (direct summation in LDS tiles, or
// radix-2 when n_a is a power of two); sc scales the output.
template <typename T>
static int axis_transform(const SpecGeom &G, const cx<T> *tw, const cx<T> *in, cx<T> *out, int a,
                          int64_t stride, int sign, T sc, hipStream_t s) {
  const int n = G.n[a];
  const int64_t total = G.S * G.nt * G.nc;
  const int64_t outer = total / ((int64_t)n * stride);
  int ti = (int)(stride < 2048 / n ? stride : 2048 / n);
  if (ti < 1) ti = 1;
  while (stride % ti) ti--;
  const int ntq = (int)(stride / ti);
  const size_t sh = ((size_t)n * ti + n) * sizeof(cx<T>);
  if ((n & (n - 1)) == 0 && (ti & (ti - 1)) == 0) {
    int logn = 0, lti = 0;
    while ((1 << logn) < n) logn++;
    while ((1 << lti) < ti) lti++;
    fft_axis<T><<<(unsigned)(outer * ntq), 256, sh, s>>>(in, out, n, logn, stride, lti, ntq, sign, sc,
                                                        tw + G.tw_off[a]);
  } else {
    dft_axis<T><<<(unsigned)(outer * ntq), 256, sh, s>>>(in, out, n, stride, ti, ntq, sign, sc,
                                                        tw + G.tw_off[a]);
  }
  DST_LAUNCHED();
  return 0;
}

template <typename T>
static int pc_setup(Precond &P, const dirac_st_bsr *A, int kind, double vbar, unsigned char *spec,
                    hipStream_t s, int slabs = 1) {
  P.kind = kind;
  P.slabs = kind == DIRAC_ST_PC_TIME_SLABS ? slabs : 1;
  P.prec = sizeof(T) == 8 ? 64 : 32;
  P.A = A;
  if (kind == DIRAC_ST_PC_BLOCK_JACOBI) {
    DST_CHECK((sizeof(T) == 8 ? A->bjinv64 : A->bjinv32) != nullptr,
              "block-Jacobi preconditioner needs bjinv%d", P.prec);
  }
  if (line_kind(kind)) return line_setup_host<T>(P, A, spec, s);
  if (kind != DIRAC_ST_PC_SPECTRAL) return 0;
  P.spec = spec;
  P.SL = spec_layout(&A->prob, P.prec);
  spec_geom(&A->prob, vbar, P.G);
  if (int rc = spec_twiddles(P.G, spec, P.SL, s)) return rc;
  P.piv_pending = true;
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
    // forward transforms over every spatial axis (v -> z, then in place),
    // block elimination along time per mode, inverse transforms
    for (int pass = 0; pass < 2; pass++) {
      int64_t stride = G.nc;
      for (int a = 1; a <= G.d; a++) {
        const bool first = (pass == 0 && a == 1);
        const bool last = (pass == 1 && a == G.d);
        const T sc = last ? (T)(scale / (double)G.S) : (T)1;
        if (int rc = axis_transform<T>(G, tw, first ? v : z, z, a, stride, pass == 0 ? -1 : 1, sc, s))
          return rc;
        stride *= G.n[a];
      }
      if (pass == 0) {
        const unsigned g = (unsigned)((G.S + 63) / 64);
        const double2 *tw64 = (const double2 *)(P.spec + P.SL.tw64);
        cx<T> *piv = (cx<T> *)(P.spec + P.SL.piv);
        auto thomas = [&](auto setup) {
          constexpr bool SU = decltype(setup)::value;
          if (G.d == 1)
            spectral_thomas<T, 2, 1, SU><<<g, 64, 0, s>>>(G, tw64, piv, z);
          else if (G.d == 2)
            spectral_thomas<T, 2, 2, SU><<<g, 64, 0, s>>>(G, tw64, piv, z);
          else
            spectral_thomas<T, 4, 3, SU><<<g, 64, 0, s>>>(G, tw64, piv, z);
        };
        if (P.piv_pending) {
          thomas(std::true_type{});
          P.piv_pending = false;
        } else {
          thomas(std::false_type{});
        }
        DST_LAUNCHED();
      }
    }
    return 0;
  }
  if (line_kind(P.kind)) {
    const SpecGeom &G = P.G;
    const LineLayout &L = P.LL;
    const bool dbl = sizeof(T) == 8;
    const cx<T> *Qm = (const cx<T> *)(P.line + (dbl ? L.q64 : L.q32));
    const cx<T> *Wm = (const cx<T> *)(P.line + (dbl ? L.w64 : L.w32));
    cx<T> *b1 = (cx<T> *)(P.line + L.buf), *b2 = (cx<T> *)(P.line + L.buf2);
    const int64_t ncol = G.S * G.nc;
    // b1 = Q v along time, per slab
    tgemm<T><<<dim3((unsigned)((ncol + 63) / 64), (unsigned)(L.pm / 64), (unsigned)L.slabs), 256, 0, s>>>(
        Qm, L.pk, v, b1, L.tl, ncol, (T)1);
    DST_LAUNCHED();
    // transverse DFTs, slowest axis first, ping-pong b1 <-> b2
    auto transverse = [&](int a, bool inverse, const cx<T> *in, cx<T> *out) -> int {
      int64_t cols = G.nc, batches = G.nt;
      for (int q = 1; q < a; q++) cols *= G.n[q];
      for (int q = a + 1; q <= G.d; q++) batches *= G.n[q];
      const cx<T> *F = (const cx<T> *)(P.line + (inverse ? (dbl ? L.fi64[a] : L.fi32[a])
                                                          : (dbl ? L.f64[a] : L.f32[a])));
      tgemm<T><<<dim3((unsigned)((cols + 63) / 64), (unsigned)(L.dpm[a] / 64), (unsigned)batches), 256, 0,
                 s>>>(F, L.dpk[a], in, out, G.n[a], cols, (T)1);
      DST_LAUNCHED();
      return 0;
    };
    cx<T> *cur = b1, *oth = b2;
    for (int a = G.d; a >= 2; a--) {
      if (int rc = transverse(a, false, cur, oth)) return rc;
      std::swap(cur, oth);
    }
    const unsigned gl = (unsigned)((L.lines + 63) / 64);
    const cx<T> *fac = (const cx<T> *)(P.line + L.fac), *lined = (const cx<T> *)(P.line + L.lined);
    const bool staged = L.lines >= kLineStagedMin;
    if (G.nc == 2) {
      if (staged) line_solve<T, 2><<<gl, 64, 0, s>>>(fac, lined, cur, G.n[1], L.lines);
      else line_solve_pt<T, 2><<<gl, 64, 0, s>>>(fac, lined, cur, G.n[1], L.lines);
    } else {
      if (staged) line_solve<T, 4><<<gl, 64, 0, s>>>(fac, lined, cur, G.n[1], L.lines);
      else line_solve_pt<T, 4><<<gl, 64, 0, s>>>(fac, lined, cur, G.n[1], L.lines);
    }
    DST_LAUNCHED();
    for (int a = 2; a <= G.d; a++) {
      if (int rc = transverse(a, true, cur, oth)) return rc;
      std::swap(cur, oth);
    }
    // z = scale * W cur along time, per slab
    tgemm<T><<<dim3((unsigned)((ncol + 63) / 64), (unsigned)(L.pm / 64), (unsigned)L.slabs), 256, 0, s>>>(
        Wm, L.pk, cur, z, L.tl, ncol, (T)scale);
    DST_LAUNCHED();
    return 0;
  }
  set_error("no preconditioner to apply");
  return DIRAC_ST_EINVAL;
}

}  // namespace dst
