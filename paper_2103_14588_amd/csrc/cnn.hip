// cnn.hip -- host side of the learned preconditioner network: workspace
// layout, forward / backward / Adam training step, and the C ABI entry points.
#include <cstring>

#include "cnn.hpp"
#include "nn_host.hpp"

namespace dst {

static Grid3 make_grid(int nt, int ny, int nx) {
  Grid3 g;
  g.nt = nt;
  g.ny = ny;
  g.nx = nx;
  g.tiles_t = (nt + TT - 1) / TT;
  g.tiles_y = (ny + TY - 1) / TY;
  g.tiles_x = (nx + TX - 1) / TX;
  g.V = (int64_t)nt * ny * nx;
  return g;
}

static const int kCh[5] = {4, 16, 16, 16, 4};

static void layer_offsets(int l, int &poff, int &woff) {
  poff = 0;
  woff = 0;
  for (int k = 0; k < l; k++) {
    poff += 27 * kCh[k] * kCh[k + 1] + kCh[k + 1];
    woff += 27 * kCh[k] * kCh[k + 1];
  }
}

NnLayout nn_layout(int nt, int ny, int nx, bool training) {
  NnLayout L{};
  const Grid3 g = make_grid(nt, ny, nx);
  const size_t V = (size_t)g.V;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.a0 = take(V * 4 * 2);
  L.a1 = take(V * 16 * 2);
  L.a2 = take(V * 16 * 2);
  L.a3 = take(V * 16 * 2);
  L.out = take(V * 4 * 4);
  if (training) {
    L.g4 = take(V * 4 * 2);
    L.g3 = take(V * 16 * 2);
    L.g2 = take(V * 16 * 2);
    L.g1 = take(V * 16 * 2);
    L.wpart = take((size_t)kWgradBlocks * 27 * 16 * 16 * 4);
    L.bpart = take((size_t)kBiasBlocks * 16 * 4);
    L.lpart = take((size_t)kLossBlocks * 2 * 8);
    L.grad = take(kNnParams * 4);
    L.loss = take(2 * 8);
  }
  L.total = off;
  return L;
}

// Persistent convolution grid: three workgroups per compute unit of the
// 256-CU MI355X (the occupancy the kernels' registers allow; each workgroup
// walks its tiles with the halo double-buffered).  Measured at 128^3: 768
// beats 512 and 1024 by 2-7 %.
static unsigned conv_grid(const Grid3 &g) {
  const int64_t nt = (int64_t)g.tiles_t * g.tiles_y * g.tiles_x;
  constexpr int64_t cap = 768;
  return (unsigned)(nt < cap ? nt : cap);
}

template <typename T>
__global__ __launch_bounds__(256) void nn_input_k(const T *__restrict__ x, double scale,
                                                  uint16_t *__restrict__ a0, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  a0[e] = f2bf((float)((double)x[e] * scale));
}

template <typename T>
__global__ __launch_bounds__(256) void nn_output_add_k(const float *__restrict__ out, double out_scale,
                                                       T *__restrict__ z, int64_t n, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double v = (double)out[e] * out_scale;
  z[e] = (T)(accumulate ? (double)z[e] + v : v);
}

// forward pass from the input already in a0; activations kept in a1..a3, output in out
static int nn_forward_from_a0(const dirac_st_nn *net, const Grid3 &g, unsigned char *w,
                              const NnLayout &L, hipStream_t s) {
  const unsigned grid = conv_grid(g);
  int poff, woff;
  uint16_t *a0 = (uint16_t *)(w + L.a0), *a1 = (uint16_t *)(w + L.a1),
           *a2 = (uint16_t *)(w + L.a2), *a3 = (uint16_t *)(w + L.a3);
  float *out = (float *)(w + L.out);
  const float *p = net->params;
  layer_offsets(0, poff, woff);
  conv3d_mfma<4, 16, CONV_RELU><<<grid, 256, 0, s>>>(g, a0, net->w16 + woff, p + poff + 27 * 4 * 16,
                                                     nullptr, a1, nullptr);
  layer_offsets(1, poff, woff);
  conv3d_mfma<16, 16, CONV_RELU><<<grid, 256, 0, s>>>(g, a1, net->w16 + woff,
                                                      p + poff + 27 * 16 * 16, nullptr, a2, nullptr);
  layer_offsets(2, poff, woff);
  conv3d_mfma<16, 16, CONV_RELU><<<grid, 256, 0, s>>>(g, a2, net->w16 + woff,
                                                      p + poff + 27 * 16 * 16, nullptr, a3, nullptr);
  layer_offsets(3, poff, woff);
  conv3d_mfma<16, 4, CONV_F32><<<grid, 256, 0, s>>>(g, a3, net->w16 + woff, p + poff + 27 * 16 * 4,
                                                    nullptr, nullptr, out);
  DST_LAUNCHED();
  return 0;
}

// gradients of all parameters into L.grad, from the bf16 gradient of the output in g4
static int nn_backward_from_g4(const dirac_st_nn *net, const Grid3 &g, unsigned char *w,
                               const NnLayout &L, hipStream_t s) {
  const unsigned grid = conv_grid(g);
  const unsigned wg = (unsigned)kWgradBlocks;
  uint16_t *a[4] = {(uint16_t *)(w + L.a0), (uint16_t *)(w + L.a1), (uint16_t *)(w + L.a2),
                    (uint16_t *)(w + L.a3)};
  uint16_t *gg[5] = {nullptr, (uint16_t *)(w + L.g1), (uint16_t *)(w + L.g2), (uint16_t *)(w + L.g3),
                     (uint16_t *)(w + L.g4)};
  float *wpart = (float *)(w + L.wpart), *bpart = (float *)(w + L.bpart), *grad = (float *)(w + L.grad);
  for (int l = 3; l >= 0; l--) {
    int poff, woff;
    layer_offsets(l, poff, woff);
    const int ci = kCh[l], co = kCh[l + 1], nw = 27 * ci * co;
    const uint16_t *gout = gg[l + 1];
    // weight gradient of layer l: input activation a[l], output gradient g_{l+1}
    if (ci == 16 && co == 4) conv3d_wgrad<16, 4><<<wg, 256, 0, s>>>(g, a[l], gout, wpart);
    else if (ci == 16) conv3d_wgrad<16, 16><<<wg, 256, 0, s>>>(g, a[l], gout, wpart);
    else conv3d_wgrad<4, 16><<<wg, 256, 0, s>>>(g, a[l], gout, wpart);
    reduce_rows<<<(nw + kReduceCols - 1) / kReduceCols, 256, 0, s>>>(wpart, (int)wg, nw, grad + poff);
    if (co == 16) bias_grad_partial<16><<<kBiasBlocks, 256, 0, s>>>(gout, g.V, bpart);
    else bias_grad_partial<4><<<kBiasBlocks, 256, 0, s>>>(gout, g.V, bpart);
    reduce_rows<<<(co + kReduceCols - 1) / kReduceCols, 256, 0, s>>>(bpart, kBiasBlocks, co, grad + poff + nw);
    // gradient of the layer input through the convolution and the ReLU of layer l-1
    if (l > 0) {
      if (co == 4)
        conv3d_mfma<4, 16, CONV_BWD><<<grid, 256, 0, s>>>(g, gout, net->wt16 + woff, nullptr, a[l],
                                                          gg[l], nullptr);
      else
        conv3d_mfma<16, 16, CONV_BWD><<<grid, 256, 0, s>>>(g, gout, net->wt16 + woff, nullptr,
                                                           a[l], gg[l], nullptr);
    }
    DST_LAUNCHED();
  }
  return 0;
}

int nn_apply_add(const dirac_st_nn *net, int nt, int ny, int nx, const void *v, int prec,
                 double in_scale, double out_scale, void *z, int accumulate, unsigned char *work,
                 hipStream_t s) {
  const Grid3 g = make_grid(nt, ny, nx);
  const NnLayout L = nn_layout(nt, ny, nx, false);
  const int64_t n = g.V * 4;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (prec == 64)
    nn_input_k<double><<<nb, 256, 0, s>>>((const double *)v, in_scale, (uint16_t *)(work + L.a0), n);
  else
    nn_input_k<float><<<nb, 256, 0, s>>>((const float *)v, in_scale, (uint16_t *)(work + L.a0), n);
  DST_LAUNCHED();
  if (int rc = nn_forward_from_a0(net, g, work, L, s)) return rc;
  if (prec == 64)
    nn_output_add_k<double><<<nb, 256, 0, s>>>((const float *)(work + L.out), out_scale,
                                               (double *)z, n, accumulate);
  else
    nn_output_add_k<float><<<nb, 256, 0, s>>>((const float *)(work + L.out), out_scale,
                                              (float *)z, n, accumulate);
  DST_LAUNCHED();
  return 0;
}

static int check_net(const dirac_st_nn *net, bool training) {
  DST_CHECK(net && net->params && net->w16 && net->wt16, "network arrays are NULL");
  DST_CHECK(!training || (net->adam_m && net->adam_v), "training needs the Adam state");
  return 0;
}

static int check_grid(int nt, int ny, int nx) {
  DST_CHECK(nt >= 1 && ny >= 3 && nx >= 3, "grid must be nt >= 1, ny >= 3, nx >= 3");
  DST_CHECK((int64_t)nt * ny * nx < (int64_t)1 << 31, "grid too large");
  return 0;
}

}  // namespace dst

using namespace dst;

extern "C" size_t dirac_st_nn_param_count(void) { return kNnParams; }

extern "C" size_t dirac_st_nn_workspace_bytes(int32_t nt, int32_t ny, int32_t nx, int32_t training) {
  if (nt < 1 || ny < 1 || nx < 1) return 0;
  return nn_layout(nt, ny, nx, training != 0).total;
}

extern "C" int dirac_st_nn_pack(const dirac_st_nn *net, void *stream) {
  clear_error();
  if (int rc = check_net(net, false)) return rc;
  pack_weights<<<(kNnParams + 255) / 256, 256, 0, (hipStream_t)stream>>>(net->params, net->w16,
                                                                          net->wt16);
  DST_LAUNCHED();
  return DIRAC_ST_OK;
}

extern "C" int dirac_st_nn_forward(const dirac_st_nn *net, int32_t nt, int32_t ny, int32_t nx,
                                   const float *in, double in_scale, float *out, void *work,
                                   size_t work_bytes, void *stream) {
  clear_error();
  if (int rc = check_net(net, false)) return rc;
  if (int rc = check_grid(nt, ny, nx)) return rc;
  DST_CHECK(in && out && work, "in, out and work must be set");
  const NnLayout L = nn_layout(nt, ny, nx, false);
  if (work_bytes < L.total) {
    set_error("workspace too small: %zu < %zu", work_bytes, L.total);
    return DIRAC_ST_ENOSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  const Grid3 g = make_grid(nt, ny, nx);
  unsigned char *w = (unsigned char *)work;
  const int64_t n = g.V * 4;
  nn_input_k<float><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, in_scale, (uint16_t *)(w + L.a0), n);
  DST_LAUNCHED();
  if (int rc = nn_forward_from_a0(net, g, w, L, s)) return rc;
  DST_HIP(hipMemcpyAsync(out, w + L.out, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  return DIRAC_ST_OK;
}

extern "C" int dirac_st_nn_backward(const dirac_st_nn *net, int32_t nt, int32_t ny, int32_t nx,
                                    const float *in, double in_scale, const float *dout, float *grad,
                                    void *work, size_t work_bytes, void *stream) {
  clear_error();
  if (int rc = check_net(net, false)) return rc;
  if (int rc = check_grid(nt, ny, nx)) return rc;
  DST_CHECK(in && dout && grad && work, "in, dout, grad and work must be set");
  const NnLayout L = nn_layout(nt, ny, nx, true);
  if (work_bytes < L.total) {
    set_error("workspace too small: %zu < %zu", work_bytes, L.total);
    return DIRAC_ST_ENOSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  const Grid3 g = make_grid(nt, ny, nx);
  unsigned char *w = (unsigned char *)work;
  const int64_t n = g.V * 4;
  const unsigned nb = (unsigned)((n + 255) / 256);
  nn_input_k<float><<<nb, 256, 0, s>>>(in, in_scale, (uint16_t *)(w + L.a0), n);
  DST_LAUNCHED();
  if (int rc = nn_forward_from_a0(net, g, w, L, s)) return rc;
  nn_input_k<float><<<nb, 256, 0, s>>>(dout, 1.0, (uint16_t *)(w + L.g4), n);
  DST_LAUNCHED();
  if (int rc = nn_backward_from_g4(net, g, w, L, s)) return rc;
  DST_HIP(hipMemcpyAsync(grad, w + L.grad, kNnParams * sizeof(float), hipMemcpyDeviceToDevice, s));
  return DIRAC_ST_OK;
}

extern "C" int dirac_st_nn_train_step(dirac_st_nn *net, int32_t nt, int32_t ny, int32_t nx,
                                      const float *in, const float *target, float lr,
                                      double *loss_out, void *work, size_t work_bytes,
                                      void *stream) {
  clear_error();
  if (int rc = check_net(net, true)) return rc;
  if (int rc = check_grid(nt, ny, nx)) return rc;
  DST_CHECK(in && target && work, "in, target and work must be set");
  const NnLayout L = nn_layout(nt, ny, nx, true);
  if (work_bytes < L.total) {
    set_error("workspace too small: %zu < %zu", work_bytes, L.total);
    return DIRAC_ST_ENOSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  const Grid3 g = make_grid(nt, ny, nx);
  unsigned char *w = (unsigned char *)work;
  const int64_t n = g.V * 4;
  const unsigned nb = (unsigned)((n + 255) / 256);
  nn_input_k<float><<<nb, 256, 0, s>>>(in, 1.0, (uint16_t *)(w + L.a0), n);
  DST_LAUNCHED();
  if (int rc = nn_forward_from_a0(net, g, w, L, s)) return rc;
  const float *out = (const float *)(w + L.out);
  double *lpart = (double *)(w + L.lpart), *loss = (double *)(w + L.loss);
  loss_partial<<<kLossBlocks, 256, 0, s>>>(out, target, n, lpart);
  loss_final<<<1, 64, 0, s>>>(lpart, kLossBlocks, loss);
  loss_grad<<<nb, 256, 0, s>>>(out, target, loss, n, (uint16_t *)(w + L.g4));
  DST_LAUNCHED();
  if (int rc = nn_backward_from_g4(net, g, w, L, s)) return rc;
  net->step += 1;
  adam_step<<<(kNnParams + 255) / 256, 256, 0, s>>>(net->params, net->adam_m, net->adam_v,
                                                    (const float *)(w + L.grad), kNnParams, lr, 0.9f,
                                                    0.999f, 1e-8f, net->step);
  pack_weights<<<(kNnParams + 255) / 256, 256, 0, s>>>(net->params, net->w16, net->wt16);
  DST_LAUNCHED();
  if (loss_out) DST_HIP(hipMemcpyAsync(loss_out, loss, sizeof(double), hipMemcpyDeviceToDevice, s));
  return DIRAC_ST_OK;
}
