// cnn.hpp -- kernels of the learned preconditioner network.
//
// Network: 3x3x3 convolutions over the spacetime grid [tau][y][x] of a 2+1D
// spinor field, channels 4 -> 16 -> 16 -> 16 -> 4 (real/imaginary parts of the
// two spinor components in and out), ReLU between layers, periodic padding in
// space and zero padding in time.  Activations are channels-last bfloat16
// [voxel][c]; weights are bfloat16 [tap][cin][cout] (tap = (dt+1)*9 +
// (dy+1)*3 + (dx+1)); accumulation is FP32 on the matrix cores
// (v_mfma_f32_16x16x16_bf16); biases, master weights, the loss and Adam are FP32.
//
// Convolution as an implicit GEMM: for 16 output voxels (one MFMA row tile)
// and 16 output channels the K dimension runs over (tap, input channel).  A
// workgroup owns a 4 x 4 x 16 voxel tile (one tau slice per wavefront, one
// y-row of 16 x per MFMA tile) and stages its halo 6 x 6 x 18 in LDS.
// Backward data is the same kernel with the taps flipped and cin/cout swapped;
// backward weights is an MFMA reduction over voxels (K = voxels).
#pragma once

#include <cstdint>

#include "common.hpp"

namespace dst {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kNnParams = 17332;
constexpr int TT = 4, TY = 4, TX = 16;       // voxel tile (256 voxels)
constexpr int HT = TT + 2, HY = TY + 2, HX = TX + 2;

// round to nearest even bfloat16 (finite inputs)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

struct Grid3 {
  int nt, ny, nx;
  int tiles_t, tiles_y, tiles_x;
  int64_t V;
};

// tile index -> origin; halo voxel (a, b, c) -> global voxel index or -1
__device__ inline void tile_origin(const Grid3 &g, int64_t tile, int &t0, int &y0, int &x0) {
  const int tx = (int)(tile % g.tiles_x);
  const int64_t r = tile / g.tiles_x;
  const int ty = (int)(r % g.tiles_y);
  const int tt = (int)(r / g.tiles_y);
  t0 = tt * TT;
  y0 = ty * TY;
  x0 = tx * TX;
}

__device__ inline int64_t halo_voxel(const Grid3 &g, int t0, int y0, int x0, int a, int b, int c) {
  const int t = t0 - 1 + a;
  if (t < 0 || t >= g.nt) return -1;
  int y = y0 - 1 + b, x = x0 - 1 + c;
  y = (y % g.ny + g.ny) % g.ny;
  x = (x % g.nx + g.nx) % g.nx;
  return ((int64_t)t * g.ny + y) * g.nx + x;
}

enum ConvMode { CONV_RELU = 0, CONV_F32 = 1, CONV_BWD = 2 };

// out = conv(in, W) (+ bias) with the epilogue of MODE:
//   CONV_RELU: bf16(relu(acc + bias))              -> out16 [V][COUT]
//   CONV_F32 : acc + bias (FP32)                     -> out32 [V][COUT]
//   CONV_BWD : bf16(acc) where mask[v][co] > 0, else 0 -> out16 (ReLU adjoint)
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void conv3d_mfma(Grid3 g, const uint16_t *__restrict__ in,
                                                   const uint16_t *__restrict__ W,
                                                   const float *__restrict__ bias,
                                                   const uint16_t *__restrict__ mask,
                                                   uint16_t *__restrict__ out16,
                                                   float *__restrict__ out32) {
  static_assert(CIN == 4 || CIN == 16, "cin");
  static_assert(COUT == 4 || COUT == 16, "cout");
  constexpr int KSTEPS = CIN == 16 ? 27 : 7;  // MFMAs per output tile
  __shared__ __attribute__((aligned(16))) uint16_t halo[HT * HY * HX * CIN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mrow = lane & 15, kg = lane >> 4;
  // B operands for this lane, all K steps: W[tap][ci][co], co = lane % 16
  s4v bw[KSTEPS];
#pragma unroll
  for (int s = 0; s < KSTEPS; s++) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      int tap, ci;
      if (CIN == 16) {
        tap = s;
        ci = 4 * kg + i;
      } else {
        tap = 4 * s + kg;
        ci = i;
      }
      const int co = mrow;
      short v = 0;
      if (tap < 27 && co < COUT) v = (short)W[(tap * CIN + ci) * COUT + co];
      bw[s][i] = v;
    }
  }
  const int64_t ntiles = (int64_t)g.tiles_t * g.tiles_y * g.tiles_x;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int t0, y0, x0;
    tile_origin(g, tile, t0, y0, x0);
    __syncthreads();
    // stage the halo: CIN bf16 per voxel, zero outside the time range
    for (int hv = threadIdx.x; hv < HT * HY * HX; hv += 256) {
      const int c = hv % HX, b = (hv / HX) % HY, a = hv / (HX * HY);
      const int64_t vox = halo_voxel(g, t0, y0, x0, a, b, c);
      uint16_t *dst = halo + hv * CIN;
      if (CIN == 16) {
        uint4 q0 = make_uint4(0, 0, 0, 0), q1 = q0;
        if (vox >= 0) {
          const uint4 *src = reinterpret_cast<const uint4 *>(in + vox * 16);
          q0 = src[0];
          q1 = src[1];
        }
        reinterpret_cast<uint4 *>(dst)[0] = q0;
        reinterpret_cast<uint4 *>(dst)[1] = q1;
      } else {
        uint2 q = make_uint2(0, 0);
        if (vox >= 0) q = *reinterpret_cast<const uint2 *>(in + vox * 4);
        *reinterpret_cast<uint2 *>(dst) = q;
      }
    }
    __syncthreads();
    const int tl = wave;  // tau within tile
#pragma unroll
    for (int r = 0; r < TY; r++) {
      f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KSTEPS; s++) {
        int tap, c0;
        if (CIN == 16) {
          tap = s;
          c0 = 4 * kg;
        } else {
          tap = 4 * s + kg;
          c0 = 0;
        }
        s4v a = {0, 0, 0, 0};
        if (tap < 27) {
          const int dt = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
          const int hv = ((tl + 1 + dt) * HY + (r + 1 + dy)) * HX + (mrow + 1 + dx);
          a = *reinterpret_cast<const s4v *>(halo + hv * CIN + c0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[s], acc, 0, 0, 0);
      }
      // D[m = 4 kg + i][n = lane % 16]: voxel x = x0 + 4 kg + i, channel co
      const int co = mrow;
      const int t = t0 + tl, y = y0 + r;
      if (co < COUT && t < g.nt && y < g.ny) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int x = x0 + 4 * kg + i;
          if (x >= g.nx) continue;
          const int64_t vox = ((int64_t)t * g.ny + y) * g.nx + x;
          float v = acc[i];
          if (MODE == CONV_RELU) {
            v += bias[co];
            // written so that NaN propagates (a broken network must show)
            out16[vox * COUT + co] = f2bf(v <= 0.f ? 0.f : v);
          } else if (MODE == CONV_F32) {
            out32[vox * COUT + co] = v + bias[co];
          } else {
            const float mk = bf2f(mask[vox * COUT + co]);
            out16[vox * COUT + co] = f2bf(mk > 0.f ? v : 0.f);
          }
        }
      }
    }
  }
}

// Partial weight gradients dW[tap][ci][co] = sum_p act[p + tap][ci] gout[p][co]
// over the tiles a workgroup visits; one FP32 row of 27*CIN*COUT per workgroup
// (written in full, zeros included).  MFMA rows = (tap, ci), columns = co,
// K = voxels (16 per MFMA).  Wavefront w owns row tiles w, w+4, ...
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv3d_wgrad(Grid3 g, const uint16_t *__restrict__ act,
                                                    const uint16_t *__restrict__ gout,
                                                    float *__restrict__ partial) {
  constexpr int NROWT = CIN == 16 ? 27 : 7;   // row tiles of 16 (tap, ci) rows
  constexpr int PERW = (NROWT + 3) / 4;        // row tiles per wavefront
  __shared__ __attribute__((aligned(16))) uint16_t halo[HT * HY * HX * CIN];
  __shared__ __attribute__((aligned(16))) uint16_t gt[TT * TY * TX * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mrow = lane & 15, kg = lane >> 4;
  f4v acc[PERW];
#pragma unroll
  for (int q = 0; q < PERW; q++) acc[q] = {0.f, 0.f, 0.f, 0.f};
  const int64_t ntiles = (int64_t)g.tiles_t * g.tiles_y * g.tiles_x;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int t0, y0, x0;
    tile_origin(g, tile, t0, y0, x0);
    __syncthreads();
    for (int hv = threadIdx.x; hv < HT * HY * HX; hv += 256) {
      const int c = hv % HX, b = (hv / HX) % HY, a = hv / (HX * HY);
      const int64_t vox = halo_voxel(g, t0, y0, x0, a, b, c);
      uint16_t *dst = halo + hv * CIN;
      if (CIN == 16) {
        uint4 q0 = make_uint4(0, 0, 0, 0), q1 = q0;
        if (vox >= 0) {
          const uint4 *src = reinterpret_cast<const uint4 *>(act + vox * 16);
          q0 = src[0];
          q1 = src[1];
        }
        reinterpret_cast<uint4 *>(dst)[0] = q0;
        reinterpret_cast<uint4 *>(dst)[1] = q1;
      } else {
        uint2 q = make_uint2(0, 0);
        if (vox >= 0) q = *reinterpret_cast<const uint2 *>(act + vox * 4);
        *reinterpret_cast<uint2 *>(dst) = q;
      }
    }
    // output-gradient tile [voxel][16] (channels >= COUT and voxels outside the grid are 0)
    {
      const int v = threadIdx.x;  // 256 voxels, one per thread
      const int x = v % TX, y = (v / TX) % TY, t = v / (TX * TY);
      const int gx = x0 + x, gy = y0 + y, gtt = t0 + t;
      const bool ok = gx < g.nx && gy < g.ny && gtt < g.nt;
      const int64_t vox = ((int64_t)gtt * g.ny + gy) * g.nx + gx;
#pragma unroll
      for (int c = 0; c < 16; c++) gt[v * 16 + c] = (ok && c < COUT) ? gout[vox * COUT + c] : (uint16_t)0;
    }
    __syncthreads();
    // K loop over the tile's voxels in chunks of 16 (one y-row of x)
    for (int kc = 0; kc < TT * TY; kc++) {
      const int tl = kc / TY, r = kc % TY;
      // B[k = voxel][n = co]: voxels 4 kg + i of this row, channel mrow
      s4v bb;
#pragma unroll
      for (int i = 0; i < 4; i++) bb[i] = (short)gt[(kc * TX + 4 * kg + i) * 16 + mrow];
#pragma unroll
      for (int q = 0; q < PERW; q++) {
        const int rt = wave + 4 * q;
        if (rt >= NROWT) continue;
        // A[m = row][k = voxel]: row = (tap, ci)
        int tap, ci;
        if (CIN == 16) {
          tap = rt;
          ci = mrow;
        } else {
          tap = 4 * rt + mrow / 4;
          ci = mrow % 4;
        }
        s4v aa = {0, 0, 0, 0};
        if (tap < 27) {
          const int dt = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
#pragma unroll
          for (int i = 0; i < 4; i++) {
            const int hv = ((tl + 1 + dt) * HY + (r + 1 + dy)) * HX + (4 * kg + i + 1 + dx);
            aa[i] = (short)halo[hv * CIN + ci];
          }
        }
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aa, bb, acc[q], 0, 0, 0);
      }
    }
  }
  // write this workgroup's partial: D[m = 4 kg + i][n = mrow]
  float *dst = partial + (int64_t)blockIdx.x * (27 * CIN * COUT);
#pragma unroll
  for (int q = 0; q < PERW; q++) {
    const int rt = wave + 4 * q;
    if (rt >= NROWT) continue;
    const int co = mrow;
    if (co >= COUT) continue;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int m = 4 * kg + i;
      int tap, ci;
      if (CIN == 16) {
        tap = rt;
        ci = m;
      } else {
        tap = 4 * rt + m / 4;
        ci = m % 4;
      }
      if (tap < 27) dst[(tap * CIN + ci) * COUT + co] = acc[q][i];
    }
  }
}

// partial[b][c] = sum over the voxels of workgroup b's grid-stride range of g[v][c]
template <int C>
__global__ __launch_bounds__(256) void bias_grad_partial(const uint16_t *__restrict__ gout,
                                                         int64_t V, float *__restrict__ partial) {
  __shared__ float red[256][C];
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; c++) acc[c] = 0.f;
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256)
#pragma unroll
    for (int c = 0; c < C; c++) acc[c] += bf2f(gout[v * C + c]);
#pragma unroll
  for (int c = 0; c < C; c++) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  if (threadIdx.x < C) {
    float s = 0.f;
    for (int t = 0; t < 256; t++) s += red[t][threadIdx.x];
    partial[(int64_t)blockIdx.x * C + threadIdx.x] = s;
  }
}

// out[j] = sum_b partial[b][j] (fixed order), j < m
__global__ __launch_bounds__(256) void reduce_rows(const float *__restrict__ partial, int nb, int m,
                                                   float *__restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int b = 0; b < nb; b++) s += partial[(int64_t)b * m + j];
  out[j] = (float)s;
}

// a0 = bf16(x * s) for complex64 input viewed as [V][4] floats
__global__ __launch_bounds__(256) void nn_input(const float *__restrict__ x, const double *scale,
                                                uint16_t *__restrict__ a0, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  a0[e] = f2bf((float)((double)x[e] * scale[0]));
}

// loss partials: num = sum (out - t)^2, den = sum t^2 (FP64 per block)
__global__ __launch_bounds__(256) void loss_partial(const float *__restrict__ out,
                                                    const float *__restrict__ tgt, int64_t n,
                                                    double *__restrict__ partial) {
  __shared__ double sn[256], sd[256];
  double a = 0.0, d = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const double df = (double)out[e] - tgt[e];
    a += df * df;
    d += (double)tgt[e] * tgt[e];
  }
  sn[threadIdx.x] = a;
  sd[threadIdx.x] = d;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sn[threadIdx.x] += sn[threadIdx.x + w];
      sd[threadIdx.x] += sd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sn[0];
    partial[2 * blockIdx.x + 1] = sd[0];
  }
}

// loss[0] = num/den over the partials (one thread)
__global__ void loss_final(const double *__restrict__ partial, int nb, double *__restrict__ loss) {
  if (threadIdx.x != 0) return;
  double a = 0.0, d = 0.0;
  for (int b = 0; b < nb; b++) {
    a += partial[2 * b];
    d += partial[2 * b + 1];
  }
  loss[0] = d > 0.0 ? a / d : 0.0;
  loss[1] = d;
}

// dL/dout = 2 (out - t) / den, rounded to bf16 (the first back-propagated gradient)
__global__ __launch_bounds__(256) void loss_grad(const float *__restrict__ out,
                                                 const float *__restrict__ tgt,
                                                 const double *__restrict__ loss, int64_t n,
                                                 uint16_t *__restrict__ g) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double den = loss[1];
  g[e] = f2bf((float)(2.0 * ((double)out[e] - tgt[e]) / den));
}

// Adam on the FP32 master parameters (bias-corrected, step >= 1)
__global__ __launch_bounds__(256) void adam_step(float *__restrict__ p, float *__restrict__ m,
                                                 float *__restrict__ v,
                                                 const float *__restrict__ grad, int n, float lr,
                                                 float b1, float b2, float eps, int step) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// bf16 copies of the weights: forward layout W[tap][ci][co] and the flipped,
// transposed layout Wt[tap'][co][ci] = W[26 - tap'][ci][co] used by backward data.
__global__ __launch_bounds__(256) void pack_weights(const float *__restrict__ p,
                                                    uint16_t *__restrict__ w16,
                                                    uint16_t *__restrict__ wt16) {
  const int CH[5] = {4, 16, 16, 16, 4};
  const int i = blockIdx.x * 256 + threadIdx.x;
  int off = 0, woff = 0;
  for (int l = 0; l < 4; l++) {
    const int ci = CH[l], co = CH[l + 1], nw = 27 * ci * co;
    if (i >= off && i < off + nw) {
      const int k = i - off;
      const int tap = k / (ci * co), c = (k / co) % ci, o = k % co;
      const uint16_t b = f2bf(p[i]);
      w16[woff + k] = b;
      wt16[woff + ((26 - tap) * co + o) * ci + c] = b;
      return;
    }
    off += nw + co;
    woff += nw;
  }
}

}  // namespace dst
