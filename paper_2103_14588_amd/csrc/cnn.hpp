// cnn.hpp -- kernels of the learned preconditioner network.
//
// Network: 3x3x3 convolutions over the spacetime grid [tau][y][x] of a 2+1D
// spinor field, channels 4 -> 16 -> 16 -> 16 -> 4 (real/imaginary parts of the
// two spinor components in and out), ReLU between layers, periodic padding in
// space and zero padding in time.  Activations are channels-last bfloat16
// [voxel][c]; weights are bfloat16 [tap][cin][cout] (tap = (dt+1)*9 +
// (dy+1)*3 + (dx+1)); accumulation is FP32 on the matrix cores; biases,
// master weights, the loss and Adam are FP32.
//
// Convolution as an implicit GEMM (v_mfma_f32_16x16x32_bf16): for 16 output
// voxels (one MFMA row tile) and 16 output channels the K dimension runs over
// (tap, input channel), 32 at a time.  A persistent workgroup walks 4 x 4 x 16
// voxel tiles (one tau slice per wavefront, one y-row of 16 x per MFMA tile)
// with the 6 x 6 x 18 halo double-buffered in LDS in a chunk-planar layout
// (16 lanes read 128 contiguous bytes), and stores through a per-wavefront
// LDS transpose.
// Backward data is the same kernel with the taps flipped and cin/cout swapped;
// backward weights is an MFMA reduction over voxels (K = voxels, 32 at a time)
// from channel-major, x-shifted LDS copies of its operands.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace dst {

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

// tile index -> origin; halo voxel (a, b, c) -> global voxel index or -1.
// Tile counts stay far below 2^31 (a grid of 2^31 tiles would need terabytes
// of activations), so tile arithmetic is 32-bit.
__device__ inline void tile_origin(const Grid3 &g, int tile, int &t0, int &y0, int &x0) {
  const int tx = tile % g.tiles_x;
  const int r = tile / g.tiles_x;
  const int ty = r % g.tiles_y;
  const int tt = r / g.tiles_y;
  t0 = tt * TT;
  y0 = ty * TY;
  x0 = tx * TX;
}

// periodic wrap of a coordinate in [-1, n + 16]: one add, a few subtractions
// only on axes shorter than the tile
__device__ inline int wrap_axis(int v, int n) {
  v += v < 0 ? n : 0;
  while (v >= n) v -= n;
  return v;
}

__device__ inline int64_t halo_voxel(const Grid3 &g, int t0, int y0, int x0, int a, int b, int c) {
  const int t = t0 - 1 + a;
  if (t < 0 || t >= g.nt) return -1;
  const int y = wrap_axis(y0 - 1 + b, g.ny), x = wrap_axis(x0 - 1 + c, g.nx);
  return ((int64_t)t * g.ny + y) * g.nx + x;
}

enum ConvMode { CONV_RELU = 0, CONV_F32 = 1, CONV_BWD = 2 };

typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kHaloVox = HT * HY * HX;             // 648 halo voxels per tile
constexpr int kHaloRounds = (kHaloVox + 255) / 256;  // staging rounds of 256 threads

// Halo of one tile, fetched into registers (CIN bf16 per voxel, 0 outside the
// time range): round u covers halo voxel threadIdx.x + 256 u.  Every lane
// issues the same loads (an address outside the halo or the time range is
// replaced by voxel 0 and the data zeroed), so the number of loads in flight
// is the same on every path and later waits need not drain them; bit u of
// the returned mask says whether round u's data is real (zeroed on the put).
template <int CIN>
__device__ __forceinline__ unsigned halo_fetch(const Grid3 &g, int tile, const uint16_t *__restrict__ in,
                                               uint4 (&pre)[kHaloRounds][2]) {
  unsigned okm = 0;
  int t0, y0, x0;
  tile_origin(g, tile, t0, y0, x0);
#pragma unroll
  for (int u = 0; u < kHaloRounds; u++) {
    const int hv = threadIdx.x + 256 * u;
    const int c = hv % HX, b = (hv / HX) % HY, a = hv / (HX * HY);
    int64_t vox = hv < kHaloVox ? halo_voxel(g, t0, y0, x0, a, b, c) : -1;
    okm |= vox >= 0 ? 1u << u : 0u;
    vox = vox >= 0 ? vox : 0;
    if constexpr (CIN == 16) {
      const uint4 *src = reinterpret_cast<const uint4 *>(in + vox * 16);
      pre[u][0] = src[0];
      pre[u][1] = src[1];
    } else {
      const uint2 q = *reinterpret_cast<const uint2 *>(in + vox * 4);
      pre[u][0] = make_uint4(q.x, q.y, 0, 0);
    }
  }
  return okm;
}

// LDS halo layout, chunk-planar: for every halo row (a, b) the CIN / 4 chunks
// of 4 channels (8 bytes) are planes of HX voxels,
//   element offset (((a HY + b) CIN / 4 + q) HX + c) 4,
// so 16 lanes reading one chunk of 16 consecutive voxels read 128 contiguous
// bytes (one pass over the banks) and every operand address is a per-lane
// base plus a constant.  (For CIN = 4 this is the plain [a][b][c][4] order.)
template <int CIN>
__device__ __forceinline__ int halo_off(int a, int b, int q, int c) {
  return (((a * HY + b) * (CIN / 4) + q) * HX + c) * 4;
}

template <int CIN>
__device__ __forceinline__ void halo_put(uint16_t *buf, const uint4 (&pre)[kHaloRounds][2], unsigned okm) {
#pragma unroll
  for (int u = 0; u < kHaloRounds; u++) {
    const int hv = threadIdx.x + 256 * u;
    if (hv < kHaloVox) {
      const int c = hv % HX, b = (hv / HX) % HY, a = hv / (HX * HY);
      const uint4 z = make_uint4(0, 0, 0, 0);
      const uint4 p0 = (okm >> u) & 1 ? pre[u][0] : z, p1 = (okm >> u) & 1 ? pre[u][1] : z;
      if constexpr (CIN == 16) {
        *reinterpret_cast<uint2 *>(buf + halo_off<16>(a, b, 0, c)) = make_uint2(p0.x, p0.y);
        *reinterpret_cast<uint2 *>(buf + halo_off<16>(a, b, 1, c)) = make_uint2(p0.z, p0.w);
        *reinterpret_cast<uint2 *>(buf + halo_off<16>(a, b, 2, c)) = make_uint2(p1.x, p1.y);
        *reinterpret_cast<uint2 *>(buf + halo_off<16>(a, b, 3, c)) = make_uint2(p1.z, p1.w);
      } else {
        *reinterpret_cast<uint2 *>(buf + halo_off<4>(a, b, 0, c)) = make_uint2(p0.x, p0.y);
      }
    }
  }
}

// K = 32 slices of the implicit GEMM (v_mfma_f32_16x16x32_bf16).  Lane group
// kg = lane / 16 holds the logical k = 8 kg .. 8 kg + 7 of both operands; A
// and B pair their k-slots the same way, so the sum does not depend on the
// order the matrix core adds them in.  Logical k of step s, element i:
//   CIN 16: tap 2 s + i / 4, channel 4 kg + i % 4   (14 steps, tap 27 = 0): the
//           taps are the same in every lane, so each operand address is one
//           per-lane base plus a constant offset
//   CIN 4 : tap 8 s + 2 kg + i / 4, channel i % 4   (4 steps, taps >= 27 = 0)
template <int CIN>
struct ConvSteps {
  static constexpr int N = CIN == 16 ? 14 : 4;
};

// A operand of step s for output row r.  base = element offset of halo voxel
// (tl, 0, 0) of the current buffer plus this lane's voxel x = mrow (and, for
// CIN 16, its channel chunk kg): CIN 16 reads base + a constant per (s, r);
// CIN 4 spreads taps over the lane groups.
template <int CIN>
__device__ __forceinline__ s8v conv_a(const uint16_t *halo, int base, int s, int r, int kg) {
  typedef short s4 __attribute__((ext_vector_type(4)));
  auto at = [&](int tap) {
    const int dt = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    return *reinterpret_cast<const s4 *>(halo + base + halo_off<CIN>(1 + dt, r + 1 + dy, 0, 1 + dx));
  };
  s4 lo = {0, 0, 0, 0}, hi = lo;
  if constexpr (CIN == 16) {
    lo = at(2 * s);
    if (2 * s + 1 < 27) hi = at(2 * s + 1);
  } else {
    const int tap = 8 * s + 2 * kg;
    if (tap < 27) lo = at(tap);
    if (tap + 1 < 27) hi = at(tap + 1);
  }
  return s8v{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// out = conv(in, W) (+ bias) with the epilogue of MODE:
//   CONV_RELU: bf16(relu(acc + bias))              -> out16 [V][COUT]
//   CONV_F32 : acc + bias (FP32)                     -> out32 [V][COUT]
//   CONV_BWD : bf16(acc) where mask[v][co] > 0, else 0 -> out16 (ReLU adjoint)
// A workgroup walks its tiles with the halo double-buffered in LDS: the next
// tile's halo is fetched into registers before the current tile's MFMAs and
// written to the other buffer after them, one barrier per tile.
template <int CIN, int COUT, int MODE>
// (three wavefronts per SIMD, two for the 16-channel backward pass, whose ReLU
// masks take 16 more registers)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == CONV_BWD && CIN == 16 ? 2 : 3)))
void conv3d_mfma(Grid3 g, const uint16_t *__restrict__ in,
                                                   const uint16_t *__restrict__ W,
                                                   const float *__restrict__ bias,
                                                   const uint16_t *__restrict__ mask,
                                                   uint16_t *__restrict__ out16,
                                                   float *__restrict__ out32) {
  static_assert(CIN == 4 || CIN == 16, "cin");
  static_assert(COUT == 16 || (COUT == 4 && MODE == CONV_F32), "bf16 outputs have 16 channels");
  constexpr int NS = ConvSteps<CIN>::N;
  constexpr int HB = kHaloVox * CIN;  // elements per halo buffer
  __shared__ __attribute__((aligned(16))) uint16_t halo[2 * HB];
  // per-wavefront output transpose: 16 voxel rows of 16 bf16 channels, rows
  // EPR = 20 elements apart so that the four lane groups (4 voxels apart) of
  // a write land on disjoint LDS banks
  constexpr int EPR = 20;
  __shared__ __attribute__((aligned(16))) uint16_t ep[4][16 * EPR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mrow = lane & 15, kg = lane >> 4;
  const int ntiles = g.tiles_t * g.tiles_y * g.tiles_x;
  int tile = blockIdx.x;
  if (tile >= ntiles) return;
  // weights W[tap][ci][co] staged in the second halo buffer as Wt[co][tap][ci]
  // (taps 27.. and channels co >= COUT zero), so each lane reads its B
  // operands (co = lane % 16) in 8-byte pieces
  constexpr int WT = 32 * CIN;  // bf16 per co row
  static_assert(16 * WT <= kHaloVox * CIN, "weights fit one halo buffer");
  uint16_t *wt = halo + HB;
  for (int e = threadIdx.x; e < 16 * WT; e += 256) {
    const int co = e / WT, tap = (e % WT) / CIN, ci = e % CIN;
    wt[e] = (tap < 27 && co < COUT) ? W[(tap * CIN + ci) * COUT + co] : (uint16_t)0;
  }
  uint4 pre[kHaloRounds][2];
  halo_put<CIN>(halo, pre, halo_fetch<CIN>(g, tile, in, pre));
  __syncthreads();
  bf8v bw[NS];
  {
    typedef short s4 __attribute__((ext_vector_type(4)));
    const uint16_t *wr = wt + mrow * WT;
#pragma unroll
    for (int s = 0; s < NS; s++) {
      // same k-slots as conv_a: (tap, channel) of elements 0..3 and 4..7
      const int ta = CIN == 16 ? 2 * s : 8 * s + 2 * kg;
      const int c0 = CIN == 16 ? 4 * kg : 0;
      const s4 lo = *reinterpret_cast<const s4 *>(wr + ta * CIN + c0);
      const s4 hi = *reinterpret_cast<const s4 *>(wr + (ta + 1) * CIN + c0);
      const s8v v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      bw[s] = __builtin_bit_cast(bf8v, v);
    }
  }
  __syncthreads();  // every lane holds its weights before halo[1] is refilled
  // global loads of the epilogue (bias, ReLU mask) are issued before the next
  // tile's halo fetch: the memory counter is in order, so a wait for a load
  // issued after the fetch would also wait for the fetch
  const int co = mrow;
  float bco = (MODE != CONV_BWD && co < COUT) ? bias[co] : 0.f;
  asm volatile("" : "+v"(bco));  // wait for it here, not inside the loop
  const int xv = lane >> 1, half = lane & 1;  // epilogue store: lanes 0..31 own voxel xv, channels 8 half ..
  for (int cur = 0; tile < ntiles; tile += gridDim.x, cur ^= 1) {
    int t0, y0, x0;
    tile_origin(g, tile, t0, y0, x0);
    const int t = t0 + wave;
    uint4 mk[TY];
    if constexpr (MODE == CONV_BWD) {
#pragma unroll
      for (int r = 0; r < TY; r++) {
        mk[r] = make_uint4(0, 0, 0, 0);
        const int y = y0 + r;
        if (t < g.nt && y < g.ny && lane < 32 && x0 + xv < g.nx)
          mk[r] = *reinterpret_cast<const uint4 *>(mask + ((((int64_t)t * g.ny + y) * g.nx + x0 + xv) * 16 + 8 * half));
      }
    }
    const int next = tile + (int)gridDim.x;
    const unsigned okm = halo_fetch<CIN>(g, next < ntiles ? next : tile, in, pre);  // unconditional: fixed load count
    const int tl = wave;  // tau within tile
    // operand base of this lane in the current buffer, opaque to the
    // optimiser so that each read is the base plus an immediate offset
    // (hoisting every (s, r) address out of the tile loop would cost a
    // register each)
    int base = cur * HB + halo_off<CIN>(tl, 0, CIN == 16 ? kg : 0, mrow);
    asm volatile("" : "+v"(base));
    f4v acc[TY];
#pragma unroll
    for (int r = 0; r < TY; r++) acc[r] = {0.f, 0.f, 0.f, 0.f};
    // A operands one step ahead: the reads of step s + 1 are in flight during
    // the MFMAs of step s (the scheduling barrier keeps the compiler from
    // hoisting every step's reads, which would cost registers and occupancy)
    s8v ac[TY];
#pragma unroll
    for (int r = 0; r < TY; r++) ac[r] = conv_a<CIN>(halo, base, 0, r, kg);
#pragma unroll
    for (int s = 0; s < NS; s++) {
      s8v an[TY];
      if (s + 1 < NS) {
#pragma unroll
        for (int r = 0; r < TY; r++) an[r] = conv_a<CIN>(halo, base, s + 1, r, kg);
      }
#pragma unroll
      for (int r = 0; r < TY; r++)
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, ac[r]), bw[s], acc[r], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      if (s + 1 < NS) {
#pragma unroll
        for (int r = 0; r < TY; r++) ac[r] = an[r];
      }
    }
    // D[m = 4 kg + i][n = lane % 16] is voxel x0 + 4 kg + i, channel co: the
    // wavefront transposes each 16-voxel row through LDS so that a lane
    // stores 16 contiguous bytes of one voxel
    uint16_t *e = ep[wave];
#pragma unroll
    for (int r = 0; r < TY; r++) {
      const int y = y0 + r;
      if (t >= g.nt || y >= g.ny) continue;  // uniform over the wavefront
      const int64_t row = ((int64_t)t * g.ny + y) * g.nx;
      if constexpr (MODE == CONV_F32) {
        float *ef = reinterpret_cast<float *>(e);  // [16 voxels][4 channels]
        if (co < COUT) {
#pragma unroll
          for (int i = 0; i < 4; i++) ef[(4 * kg + i) * 4 + co] = acc[r][i] + bco;
        }
        if (lane < 16 && x0 + lane < g.nx)
          *reinterpret_cast<float4 *>(out32 + (row + x0 + lane) * 4) = reinterpret_cast<const float4 *>(ef)[lane];
      } else {
#pragma unroll
        for (int i = 0; i < 4; i++) {
          float v = acc[r][i];
          // written so that NaN propagates (a broken network must show)
          if (MODE == CONV_RELU) v = (v + bco) <= 0.f ? 0.f : v + bco;
          e[(4 * kg + i) * EPR + co] = f2bf(v);
        }
        if (lane < 32 && x0 + xv < g.nx) {
          const int64_t o = (row + x0 + xv) * 16 + 8 * half;
          const uint2 lo = *reinterpret_cast<const uint2 *>(e + xv * EPR + 8 * half);
          const uint2 hi = *reinterpret_cast<const uint2 *>(e + xv * EPR + 8 * half + 4);
          uint4 q = make_uint4(lo.x, lo.y, hi.x, hi.y);
          if constexpr (MODE == CONV_BWD) {
            // ReLU adjoint: keep the gradient where the forward activation was positive
            const uint4 m = mk[r];
            // (a bfloat16 is > 0 exactly when its bits lie in (0, 0x7F80]:
            // positive, +inf included, NaN and -0 excluded)
            auto pos = [](uint32_t b) { return b - 1u < 0x7F80u; };
            auto keep = [&](uint32_t gv, uint32_t m) {
              return (pos(m & 0xFFFFu) ? (gv & 0xFFFFu) : 0u) | (pos(m >> 16) ? (gv & 0xFFFF0000u) : 0u);
            };
            q = make_uint4(keep(q.x, m.x), keep(q.y, m.y), keep(q.z, m.z), keep(q.w, m.w));
          }
          *reinterpret_cast<uint4 *>(out16 + o) = q;
        }
      }
    }
    if (next < ntiles) halo_put<CIN>(halo + (cur ^ 1) * HB, pre, okm);
    __syncthreads();
  }
}

// Partial weight gradients dW[tap][ci][co] = sum_p act[p + tap][ci] gout[p][co]
// over the tiles a workgroup visits; one FP32 row of 27*CIN*COUT per workgroup
// (written in full, zeros included).  GEMM with M = (tap, ci), N = co (16,
// zero-padded for COUT 4) and K = voxels, 32 per v_mfma_f32_16x16x32_bf16: a
// K step covers two 16-voxel x-rows of the tile, lane group kg holding
// voxels x = 8 (kg & 1) .. + 7 of row kg >> 1 in both operands.  Both
// operands are staged channel-major so that these 8 voxels are 16 contiguous
// bytes: the output gradient as gT[co][t][y][x], the activations as three
// copies of the halo shifted by 0, 1, 2 voxels along x,
//   cp[s][ci][a][b][j] = halo[ci][a][b][j + s], j < 16,
// so that the operand of any tap (shift s = dx + 1) is one aligned 16-byte
// read.  Each channel plane is padded by 16 bytes: the 16 lanes of a read
// differ only in the channel, and unpadded planes (multiples of 128 bytes)
// would put all of them on the same LDS banks.  Row tiles: CIN 16 -> one tap (m = ci), wavefront w owns taps w, w+4,
// ...; CIN 4 -> four taps (m = 4 (tap % 4) + ci), row tile r = taps 4r..4r+3.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv3d_wgrad(Grid3 g, const uint16_t *__restrict__ act,
                                                    const uint16_t *__restrict__ gout,
                                                    float *__restrict__ partial) {
  static_assert(CIN == 4 || CIN == 16, "cin");
  static_assert(COUT == 4 || COUT == 16, "cout");
  constexpr int NROWT = CIN == 16 ? 27 : 7;   // row tiles of 16 (tap, ci) rows
  constexpr int PERW = (NROWT + 3) / 4;        // row tiles per wavefront
  constexpr int HROW = 16;                     // elements per staged x-row
  constexpr int CHS = HT * HY * HROW + 8;      // elements per channel plane (padded)
  constexpr int CP = CIN * CHS;                // elements per shifted copy
  constexpr int GS = TT * TY * TX + 8;         // elements per output-gradient plane (padded)
  __shared__ __attribute__((aligned(16))) uint16_t cp[3 * CP];
  __shared__ __attribute__((aligned(16))) uint16_t gT[16 * GS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mrow = lane & 15, kg = lane >> 4;
  // output-gradient channels >= COUT stay zero
  for (int e = threadIdx.x; e < 16 * GS; e += 256) gT[e] = 0;
  f4v acc[PERW];
#pragma unroll
  for (int q = 0; q < PERW; q++) acc[q] = {0.f, 0.f, 0.f, 0.f};
  // the next tile's activations and output gradient are fetched into
  // registers while the current tile's MFMAs run
  uint4 pre[kHaloRounds][2], pg[2];
  unsigned okm = 0;
  auto fetch_gout = [&](int tile) {
    int t0, y0, x0;
    tile_origin(g, tile, t0, y0, x0);
    const int v = threadIdx.x;
    const int x = v % TX, y = (v / TX) % TY, t = v / (TX * TY);
    const int gx = x0 + x, gy = y0 + y, gtt = t0 + t;
    const bool ok = gx < g.nx && gy < g.ny && gtt < g.nt;  // 0 outside the grid
    const int64_t vox = ok ? ((int64_t)gtt * g.ny + gy) * g.nx + gx : 0;
    if constexpr (COUT == 16) {
      const uint4 *src = reinterpret_cast<const uint4 *>(gout + vox * 16);
      pg[0] = src[0];
      pg[1] = src[1];
    } else {
      const uint2 q = *reinterpret_cast<const uint2 *>(gout + vox * 4);
      pg[0] = make_uint4(q.x, q.y, 0, 0);
      pg[1] = make_uint4(0, 0, 0, 0);
    }
    if (!ok) pg[0] = pg[1] = make_uint4(0, 0, 0, 0);
  };
  const int ntiles = g.tiles_t * g.tiles_y * g.tiles_x;
  if ((int)blockIdx.x < ntiles) {
    okm = halo_fetch<CIN>(g, blockIdx.x, act, pre);
    fetch_gout(blockIdx.x);
  }
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // the previous tile's operands are consumed
    // activations: halo voxel (a, b, c) goes to copy s at j = c - s
#pragma unroll
    for (int u = 0; u < kHaloRounds; u++) {
      const int hv = threadIdx.x + 256 * u;
      if (hv >= kHaloVox) continue;
      const int c = hv % HX, b = (hv / HX) % HY, a = hv / (HX * HY);
      const uint4 z = make_uint4(0, 0, 0, 0);
      const uint4 q0 = (okm >> u) & 1 ? pre[u][0] : z, q1 = (okm >> u) & 1 ? pre[u][1] : z;
      const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
      uint16_t v[CIN];
#pragma unroll
      for (int i = 0; i < CIN / 2; i++) {
        v[2 * i] = (uint16_t)(w[i] & 0xFFFFu);
        v[2 * i + 1] = (uint16_t)(w[i] >> 16);
      }
#pragma unroll
      for (int sft = 0; sft < 3; sft++) {
        const int j = c - sft;
        if (j < 0 || j >= HROW) continue;
#pragma unroll
        for (int ci = 0; ci < CIN; ci++) cp[sft * CP + ci * CHS + (a * HY + b) * HROW + j] = v[ci];
      }
    }
    // output gradient: voxel v of the tile (t, y, x) = (v / 64, v / 16 % 4, v % 16)
    {
      const int v = threadIdx.x;
      const uint32_t w[8] = {pg[0].x, pg[0].y, pg[0].z, pg[0].w, pg[1].x, pg[1].y, pg[1].z, pg[1].w};
#pragma unroll
      for (int i = 0; i < COUT / 2; i++) {
        gT[(2 * i) * GS + v] = (uint16_t)(w[i] & 0xFFFFu);
        gT[(2 * i + 1) * GS + v] = (uint16_t)(w[i] >> 16);
      }
    }
    __syncthreads();
    {
      const int next = tile + (int)gridDim.x;
      const int nt = next < ntiles ? next : tile;  // unconditional: fixed load count
      okm = halo_fetch<CIN>(g, nt, act, pre);
      fetch_gout(nt);
    }
    // K steps: step k covers tau slice k / 2, y-rows 2 (k % 2) and 2 (k % 2) + 1
    const int h = kg & 1;
#pragma unroll 2
    for (int k = 0; k < TT * TY / 2; k++) {
      const int t = k >> 1, y = 2 * (k & 1) + (kg >> 1);
      const bf8v bb = __builtin_bit_cast(bf8v, *reinterpret_cast<const s8v *>(
                                                   gT + mrow * GS + (t * TY + y) * TX + 8 * h));
#pragma unroll
      for (int q = 0; q < PERW; q++) {
        const int rt = wave + 4 * q;
        if (rt >= NROWT) continue;
        int tap, ci;
        if (CIN == 16) {
          tap = rt;
          ci = mrow;
        } else {
          tap = 4 * rt + (mrow >> 2);
          ci = mrow & 3;
        }
        s8v aa = {0, 0, 0, 0, 0, 0, 0, 0};
        if (tap < 27) {
          const int dt = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
          aa = *reinterpret_cast<const s8v *>(
              cp + (dx + 1) * CP + ci * CHS + ((t + 1 + dt) * HY + (y + 1 + dy)) * HROW + 8 * h);
        }
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, aa), bb, acc[q], 0, 0, 0);
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

// out[j] = sum_b partial[b][j], j < m, in a fixed order: a workgroup owns 64
// consecutive j (one per lane, coalesced rows); wavefront w sums rows
// w, w + 4, ... and the four sums are added in wavefront order
constexpr int kReduceCols = 64;
__global__ __launch_bounds__(256) void reduce_rows(const float *__restrict__ partial, int nb, int m,
                                                   float *__restrict__ out) {
  __shared__ double red[4][kReduceCols];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * kReduceCols + lane;
  double s = 0.0;
  if (j < m) {
#pragma unroll 8
    for (int b = w; b < nb; b += 4) s += partial[(int64_t)b * m + j];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < m) out[j] = (float)(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
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
