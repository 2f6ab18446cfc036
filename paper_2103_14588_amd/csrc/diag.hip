// diag.hip -- per-time-slice diagnostics of a solution: the charge of
// Sec. 4.1, the numerators of <x(t)> (Sec. 4.2) and of the transmission and
// reflection coefficients of Sec. 4.3 (eq. (klein:coeffs)), as trapezoid sums
// on the periodic uniform mesh (nodal sums times the cell volume).
#include "common.hpp"

namespace dst {

// One workgroup per time node tau = 0..n_t (slice 0 is psi0); each thread
// sums a fixed subset of nodes in index order, then the workgroup reduces in
// a fixed order (deterministic).  out[tau][0] = sum |psi|^2,
// out[tau][1] = the same over x_1 > x_split, out[tau][2 + a] = sum x_a |psi|^2.
template <int NC, int DS>
__global__ __launch_bounds__(256) void slice_moments_kernel(int n1, int n2, int64_t S,
                                                            double h1, double h2, double h3, double vol,
                                                            const double2 *__restrict__ psi0,
                                                            const double2 *__restrict__ x, double x_split,
                                                            double *__restrict__ out) {
  constexpr int K = 2 + DS;
  __shared__ double red[K][4];
  const int tau = blockIdx.x;
  const double2 *slice = tau == 0 ? psi0 : x + (int64_t)(tau - 1) * S * NC;
  const double h[3] = {h1, h2, h3};
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; k++) acc[k] = 0.0;
  for (int64_t s = threadIdx.x; s < S; s += 256) {
    double dens = 0.0;
#pragma unroll
    for (int c = 0; c < NC; c++) {
      const double2 v = slice[s * NC + c];
      dens += v.x * v.x + v.y * v.y;
    }
    int64_t r = s;
    int ia[3];
    ia[0] = (int)(r % n1);
    r /= n1;
    if (DS >= 2) {
      ia[1] = (int)(r % n2);
      r /= n2;
    }
    if (DS >= 3) ia[2] = (int)r;
    acc[0] += dens;
    if (ia[0] * h[0] > x_split) acc[1] += dens;
#pragma unroll
    for (int a = 0; a < DS; a++) acc[2 + a] += ia[a] * h[a] * dens;
  }
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; k++) {
    double v = acc[k];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    const int k = threadIdx.x;
    out[(int64_t)tau * K + k] = vol * (red[k][0] + red[k][1] + red[k][2] + red[k][3]);
  }
}

}  // namespace dst

using namespace dst;

extern "C" int dirac_st_slice_moments(const dirac_st_problem *p, const void *psi0, const void *x, double x_split,
                                      double *out, void *stream) {
  clear_error();
  DST_CHECK(p != nullptr, "problem is NULL");
  if (int rc = validate_problem(p)) return rc;
  DST_CHECK(psi0 && x && out, "psi0, x and out must be set");
  DST_CHECK(((uintptr_t)psi0 & 15) == 0 && ((uintptr_t)x & 15) == 0, "psi0, x must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int d = p->d, nt = p->n[0];
  int64_t S = 1;
  double vol = 1.0, h[3] = {1.0, 1.0, 1.0};
  for (int a = 1; a <= d; a++) {
    S *= p->n[a];
    h[a - 1] = p->len[a] / p->n[a];
    vol *= h[a - 1];
  }
  const int n1 = p->n[1], n2 = d >= 2 ? p->n[2] : 1;
  const double2 *ps = (const double2 *)psi0, *xx = (const double2 *)x;
  const unsigned g = (unsigned)(nt + 1);
  if (d == 1)
    slice_moments_kernel<2, 1><<<g, 256, 0, s>>>(n1, n2, S, h[0], h[1], h[2], vol, ps, xx, x_split, out);
  else if (d == 2)
    slice_moments_kernel<2, 2><<<g, 256, 0, s>>>(n1, n2, S, h[0], h[1], h[2], vol, ps, xx, x_split, out);
  else
    slice_moments_kernel<4, 3><<<g, 256, 0, s>>>(n1, n2, S, h[0], h[1], h[2], vol, ps, xx, x_split, out);
  DST_LAUNCHED();
  return DIRAC_ST_OK;
}
