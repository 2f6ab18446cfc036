// common.hpp -- shared helpers of the HIP library: complex arithmetic on
// double2/float2, error reporting across the C ABI, problem validation and
// mesh indexing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "dirac_st.h"

namespace dst {

// ------------------------------------------------------------ complex
template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename T> using cx = typename cplx_of<T>::type;

template <typename C> __host__ __device__ inline C mk(decltype(C::x) re, decltype(C::x) im) {
  C c;
  c.x = re;
  c.y = im;
  return c;
}
template <typename C> __host__ __device__ inline C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __host__ __device__ inline C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
template <typename C> __host__ __device__ inline C cfma(C acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
template <typename C> __host__ __device__ inline C cfma_conj(C acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
// acc - a * b
template <typename C> __host__ __device__ inline C cfms(C acc, C a, C b) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename C> __host__ __device__ inline C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

__host__ __device__ inline float2 to32(double2 a) { return mk<float2>((float)a.x, (float)a.y); }
__host__ __device__ inline double2 to64(float2 a) { return mk<double2>((double)a.x, (double)a.y); }
__host__ __device__ inline double2 to64(double2 a) { return a; }

// ------------------------------------------------------------ errors
void set_error(const char *fmt, ...);
void clear_error();

#define DST_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::dst::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                       \
      return DIRAC_ST_EHIP;                                                             \
    }                                                                                   \
  } while (0)

#define DST_LAUNCHED()                                                                        \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess) {                                                                   \
      ::dst::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                             \
      return DIRAC_ST_EHIP;                                                                   \
    }                                                                                         \
  } while (0)

#define DST_CHECK(cond, ...)          \
  do {                                \
    if (!(cond)) {                    \
      ::dst::set_error(__VA_ARGS__);  \
      return DIRAC_ST_EINVAL;         \
    }                                 \
  } while (0)

// ------------------------------------------------------------ mesh
// Validates the problem; returns 0 or sets the error and returns EINVAL.
int validate_problem(const dirac_st_problem *p);

// spatial nodes S and block rows n_t * S
int64_t spatial_nodes(const dirac_st_problem *p);
// blocks per row in time slice tau (1-based): (#time neighbours in 1..n_t) * 3^d
int blocks_per_row(const dirac_st_problem *p, int tau);
int64_t total_blocks(const dirac_st_problem *p);

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Optional timing of selected kernels with HIP events recorded around their
// launches on the launch stream (off unless dirac_st_timing(1) was called).
// kt_start returns a token (-1 when timing is off); kt_stop closes it.
int kt_start(int kind, hipStream_t s);
void kt_stop(int token, hipStream_t s);

// Rows handled by one XCD stay contiguous: hardware dispatches workgroup b to
// XCD b % 8, so logical tile = position inside that XCD's share.
// byte skew between consecutive vectors of a workspace (basis vectors and
// the like), so that streams read together do not start a power of two apart
constexpr size_t kVecSkew = 4096;

// Gamma matrices g^mu, row-major nc x nc, for d spatial dimensions.
inline void gamma_set(int d, double2 (*g)[16]) {
  for (int mu = 0; mu < 4; mu++)
    for (int q = 0; q < 16; q++) g[mu][q] = mk<double2>(0, 0);
  if (d <= 2) {
    // g0 = diag(1, -1), g1 = [[0, 1], [-1, 0]] (App. A); g2 = [[0, -i], [-i, 0]]
    g[0][0] = mk<double2>(1, 0);
    g[0][3] = mk<double2>(-1, 0);
    g[1][1] = mk<double2>(1, 0);
    g[1][2] = mk<double2>(-1, 0);
    g[2][1] = mk<double2>(0, -1);
    g[2][2] = mk<double2>(0, -1);
    return;
  }
  // Dirac representation: g0 = diag(I, -I), gk = [[0, s_k], [-s_k, 0]]
  for (int q = 0; q < 4; q++) g[0][q * 5] = mk<double2>(q < 2 ? 1 : -1, 0);
  const double2 pauli[3][4] = {
      {mk<double2>(0, 0), mk<double2>(1, 0), mk<double2>(1, 0), mk<double2>(0, 0)},
      {mk<double2>(0, 0), mk<double2>(0, -1), mk<double2>(0, 1), mk<double2>(0, 0)},
      {mk<double2>(1, 0), mk<double2>(0, 0), mk<double2>(0, 0), mk<double2>(-1, 0)}};
  for (int k = 1; k <= 3; k++)
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++) {
        double2 s = pauli[k - 1][a * 2 + b];
        g[k][a * 4 + b + 2] = s;
        g[k][(a + 2) * 4 + b] = mk<double2>(-s.x, -s.y);
      }
}

__device__ inline int64_t xcd_tile(int64_t b, int64_t nwg) {
  const int64_t x = b & 7, q = b >> 3;
  const int64_t per = nwg >> 3, rem = nwg & 7;
  return (x < rem) ? x * (per + 1) + q : rem * (per + 1) + (x - rem) * per + q;
}

}  // namespace dst
